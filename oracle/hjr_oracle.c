/*
 * hjr_oracle.c -- plain, single-threaded FP64 reference for the grid-based
 * Hamilton-Jacobi reachability safe-set solve.
 *
 * TEST INFRASTRUCTURE ONLY: the product library never links or calls it.
 * It is written for checkability, not speed: every node is evaluated on its
 * own, from its own five-point line windows, with the Hamiltonian found by
 * enumerating control and disturbance vertices.
 *
 * Method (paper Sec. II-A): the value of eq. (1) is found by iterating the
 * HJI variational inequality eq. (2) backwards in time from V = l until it
 * stops changing.  With the sign convention of hjr_oracle.h that reads
 *     V_tau = max_u min_d grad V . f(x,u,d),  then  V <- min(l, V).
 * Warm start (Sec. III-B): the same iteration started from a previous
 * converged value.  Coarse approximations (Sec. III-C): converge on a coarse
 * grid, carry the result to a finer grid, continue.  Decomposition
 * (Sec. III-A, eq. (3)): each subsystem is solved as its own problem.
 *
 * Parity pins for each function are in the test-suite; see the comments
 * there for which closed form, invariant or brute force pins which function.
 */
#include "hjr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Dynamics: the subsystem models of Sec. IV eq. (3) (x- and z-subsystems)   */
/* and Sec. V, plus a test-only product of two independent vertical models.  */
/* ------------------------------------------------------------------------ */

int orc_state_dim(int kind)
{
    switch (kind) {
    case ORC_QUAD_Z2D: return 2;
    case ORC_QUAD_X4D: return 4;
    case ORC_QUAD_X4DV: return 4;
    case ORC_DI2X2: return 4;
    default: return 0;
    }
}

int orc_num_ctrl(int kind)
{
    switch (kind) {
    case ORC_QUAD_Z2D: return 1;
    case ORC_QUAD_X4D: return 1;
    case ORC_QUAD_X4DV: return 1;
    case ORC_DI2X2: return 2;
    default: return 0;
    }
}

int orc_num_dstb(int kind)
{
    switch (kind) {
    case ORC_QUAD_Z2D: return 1;
    case ORC_QUAD_X4D: return 1;
    case ORC_QUAD_X4DV: return 1;
    case ORC_DI2X2: return 2;
    default: return 0;
    }
}

/* tan() memoised on its last argument: the node loops vary the last axis
 * fastest, so theta repeats for whole rows. */
static double memo_tan(double th)
{
    static double last_arg = 0.0, last_val = 0.0;
    static int have = 0;
    if (!have || th != last_arg) {
        last_arg = th;
        last_val = tan(th);
        have = 1;
    }
    return last_val;
}

void orc_dynamics(const orc_dyn* dyn, const double* x, const double* u,
                  const double* d, double* f)
{
    const double* p = dyn->p;
    switch (dyn->kind) {
    case ORC_QUAD_Z2D:
        /* z' = vz ; vz' = k u - g + d */
        f[0] = x[1];
        f[1] = p[0] * u[0] - p[1] + d[0];
        break;
    case ORC_QUAD_X4D:
        /* x' = vx + d ; vx' = g tan(theta) ; theta' = -d1 theta + omega ;
         * omega' = -d0 theta + n0 S */
        f[0] = x[1] + d[0];
        f[1] = p[0] * memo_tan(x[2]);
        f[2] = -p[1] * x[2] + x[3];
        f[3] = -p[2] * x[2] + p[3] * u[0];
        break;
    case ORC_QUAD_X4DV:
        /* the x rows of the 10-D model: x' = vx ; vx' = g tan(theta) + d ;
         * theta' = -d1 theta + omega ; omega' = -d0 theta + n0 S */
        f[0] = x[1];
        f[1] = p[0] * memo_tan(x[2]) + d[0];
        f[2] = -p[1] * x[2] + x[3];
        f[3] = -p[2] * x[2] + p[3] * u[0];
        break;
    case ORC_DI2X2: {
        int za = (int)p[8], va = (int)p[9], zb = (int)p[10], vb = (int)p[11];
        f[za] = x[va];
        f[va] = p[0] * u[0] - p[1] + d[0];
        f[zb] = x[vb];
        f[vb] = p[4] * u[1] - p[5] + d[1];
        break;
    }
    default:
        break;
    }
}

void orc_ctrl_box(const orc_dyn* dyn, double* lo, double* hi)
{
    const double* p = dyn->p;
    switch (dyn->kind) {
    case ORC_QUAD_Z2D:
        lo[0] = p[2];
        hi[0] = p[3];
        break;
    case ORC_QUAD_X4D:
    case ORC_QUAD_X4DV:
        lo[0] = -p[4];
        hi[0] = p[4];
        break;
    case ORC_DI2X2:
        lo[0] = p[2];
        hi[0] = p[3];
        lo[1] = p[6];
        hi[1] = p[7];
        break;
    default:
        break;
    }
}

/* Vertex number v of a box with m inputs: bit i of v picks hi for input i. */
static void box_vertex(int m, const double* lo, const double* hi, int v,
                       double* out)
{
    for (int i = 0; i < m; i++) out[i] = ((v >> i) & 1) ? hi[i] : lo[i];
}

/* Disturbance box of node idx (Sec. II-A: the disturbance set D(x) may
 * depend on the state).  With a per-node field, channel c is bounded by
 * dfield[(2c) N + idx] below and dfield[(2c + 1) N + idx] above; without
 * one, by the constant box dlo[c], dhi[c]. */
static void node_dbox(int md, const double* dlo, const double* dhi,
                      const double* dfield, int64_t N, int64_t idx,
                      double* lo, double* hi)
{
    for (int c = 0; c < md; c++) {
        if (dfield) {
            lo[c] = dfield[(int64_t)(2 * c) * N + idx];
            hi[c] = dfield[(int64_t)(2 * c + 1) * N + idx];
        } else {
            lo[c] = dlo[c];
            hi[c] = dhi[c];
        }
    }
}

double orc_hamiltonian(const orc_dyn* dyn, const double* x, const double* p,
                       const double* dlo, const double* dhi)
{
    int D = orc_state_dim(dyn->kind);
    int mu = orc_num_ctrl(dyn->kind), md = orc_num_dstb(dyn->kind);
    double ulo[4], uhi[4], u[4], d[4], f[4];
    orc_ctrl_box(dyn, ulo, uhi);
    double best = -INFINITY;
    for (int vu = 0; vu < (1 << mu); vu++) {
        box_vertex(mu, ulo, uhi, vu, u);
        double worst = INFINITY;
        for (int vd = 0; vd < (1 << md); vd++) {
            box_vertex(md, dlo, dhi, vd, d);
            orc_dynamics(dyn, x, u, d, f);
            double s = 0.0;
            for (int i = 0; i < D; i++) s += p[i] * f[i];
            if (s < worst) worst = s;
        }
        if (worst > best) best = worst;
    }
    return best;
}

/* ------------------------------------------------------------------------ */
/* Grid                                                                      */
/* ------------------------------------------------------------------------ */

static double spacing(const orc_grid* g, int axis)
{
    return (g->hi[axis] - g->lo[axis]) / (double)(g->n[axis] - 1);
}

double orc_coord(const orc_grid* g, int axis, int j)
{
    return g->lo[axis] + (double)j * spacing(g, axis);
}

static int64_t grid_size(const orc_grid* g)
{
    int64_t N = 1;
    for (int i = 0; i < g->ndim; i++) N *= g->n[i];
    return N;
}

static void unflatten(const orc_grid* g, int64_t idx, int* j)
{
    for (int i = g->ndim - 1; i >= 0; i--) {
        j[i] = (int)(idx % g->n[i]);
        idx /= g->n[i];
    }
}

static int64_t stride_of(const orc_grid* g, int axis)
{
    int64_t s = 1;
    for (int i = g->ndim - 1; i > axis; i--) s *= g->n[i];
    return s;
}

static int grid_valid(const orc_grid* g)
{
    if (g->ndim < 1 || g->ndim > 4) return 0;
    for (int i = 0; i < g->ndim; i++) {
        if (g->n[i] < 3) return 0;
        if (!(g->lo[i] < g->hi[i])) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Lax-Friedrichs bounds and time step                                       */
/* ------------------------------------------------------------------------ */

void orc_lf_alpha_field(const orc_dyn* dyn, const orc_grid* g,
                        const double* dlo, const double* dhi,
                        const double* dfield, double* alpha)
{
    int D = g->ndim;
    int mu = orc_num_ctrl(dyn->kind), md = orc_num_dstb(dyn->kind);
    double ulo[4], uhi[4], u[4], d[4], f[4], x[4], blo[2], bhi[2];
    int j[4];
    orc_ctrl_box(dyn, ulo, uhi);
    for (int i = 0; i < D; i++) alpha[i] = 0.0;
    int64_t N = grid_size(g);
    for (int64_t idx = 0; idx < N; idx++) {
        unflatten(g, idx, j);
        for (int i = 0; i < D; i++) x[i] = orc_coord(g, i, j[i]);
        node_dbox(md, dlo, dhi, dfield, N, idx, blo, bhi);
        for (int vu = 0; vu < (1 << mu); vu++) {
            box_vertex(mu, ulo, uhi, vu, u);
            for (int vd = 0; vd < (1 << md); vd++) {
                box_vertex(md, blo, bhi, vd, d);
                orc_dynamics(dyn, x, u, d, f);
                for (int i = 0; i < D; i++)
                    if (fabs(f[i]) > alpha[i]) alpha[i] = fabs(f[i]);
            }
        }
    }
}

void orc_lf_alpha(const orc_dyn* dyn, const orc_grid* g, const double* dlo,
                  const double* dhi, double* alpha)
{
    orc_lf_alpha_field(dyn, g, dlo, dhi, NULL, alpha);
}

double orc_dt(const orc_grid* g, const double* alpha, double cfl)
{
    double s = 0.0;
    for (int i = 0; i < g->ndim; i++) s += alpha[i] / spacing(g, i);
    return cfl / s;
}

/* ------------------------------------------------------------------------ */
/* Upwind derivatives                                                        */
/* ------------------------------------------------------------------------ */

/* Value at position jj in [-2, n+1] of the line v[0..n-1] (stride s), the
 * outside positions filled by linear extrapolation from the two end nodes. */
static double line_value(const double* v, int64_t s, int n, int jj)
{
    if (jj >= 0 && jj < n) return v[(int64_t)jj * s];
    double a0 = v[0], a1 = v[s];
    double b0 = v[(int64_t)(n - 1) * s], b1 = v[(int64_t)(n - 2) * s];
    if (jj == -1) return 2.0 * a0 - a1;
    if (jj == -2) return 3.0 * a0 - 2.0 * a1;
    if (jj == n) return 2.0 * b0 - b1;
    /* jj == n + 1 */
    return 3.0 * b0 - 2.0 * b1;
}

/* D^- and D^+ at the middle of the five samples w[0..4] (positions
 * j-2..j+2), spacing h.  ENO2: first divided differences at the half
 * nodes, second divided differences at the nodes, and of the two candidate
 * second differences the one of smaller magnitude; a tie takes the one
 * farther from j (both sides alike, so the scheme is mirror-symmetric). */
static void eno_point(const double* w, double h, int order, double* pm,
                      double* pp)
{
    double D1_m32 = (w[1] - w[0]) / h; /* at j - 3/2 */
    double D1_m12 = (w[2] - w[1]) / h; /* at j - 1/2 */
    double D1_p12 = (w[3] - w[2]) / h; /* at j + 1/2 */
    double D1_p32 = (w[4] - w[3]) / h; /* at j + 3/2 */
    if (order == 1) {
        *pm = D1_m12;
        *pp = D1_p12;
        return;
    }
    double D2_m1 = (D1_m12 - D1_m32) / (2.0 * h); /* at j - 1 */
    double D2_0 = (D1_p12 - D1_m12) / (2.0 * h);  /* at j */
    double D2_p1 = (D1_p32 - D1_p12) / (2.0 * h); /* at j + 1 */
    double cm = (fabs(D2_m1) <= fabs(D2_0)) ? D2_m1 : D2_0;
    double cp = (fabs(D2_p1) <= fabs(D2_0)) ? D2_p1 : D2_0;
    *pm = D1_m12 + h * cm;
    *pp = D1_p12 - h * cp;
}

void orc_line_derivs(const double* v, int n, double h, int order, double* pm,
                     double* pp)
{
    double w[5];
    for (int j = 0; j < n; j++) {
        for (int k = 0; k < 5; k++) w[k] = line_value(v, 1, n, j - 2 + k);
        eno_point(w, h, order, &pm[j], &pp[j]);
    }
}

/* L(V) at node idx. */
static double node_op(const orc_dyn* dyn, const orc_grid* g, const double* dlo,
                      const double* dhi, const double* dfield,
                      const double* alpha, int order, const double* V,
                      int64_t idx)
{
    int D = g->ndim;
    int j[4];
    double x[4], pbar[4], diss = 0.0, w[5], blo[2], bhi[2];
    unflatten(g, idx, j);
    for (int i = 0; i < D; i++) {
        int64_t s = stride_of(g, i);
        const double* line0 = V + (idx - (int64_t)j[i] * s); /* node 0 of this line */
        for (int k = 0; k < 5; k++) w[k] = line_value(line0, s, g->n[i], j[i] - 2 + k);
        double pm, pp;
        eno_point(w, spacing(g, i), order, &pm, &pp);
        pbar[i] = 0.5 * (pp + pm);
        diss += alpha[i] * 0.5 * (pp - pm);
        x[i] = orc_coord(g, i, j[i]);
    }
    node_dbox(orc_num_dstb(dyn->kind), dlo, dhi, dfield, grid_size(g), idx, blo, bhi);
    return orc_hamiltonian(dyn, x, pbar, blo, bhi) + diss;
}

void orc_spatial_op_field(const orc_dyn* dyn, const orc_grid* g,
                          const double* dlo, const double* dhi,
                          const double* dfield, const double* alpha, int order,
                          const double* V, double* L)
{
    int64_t N = grid_size(g);
    for (int64_t idx = 0; idx < N; idx++)
        L[idx] = node_op(dyn, g, dlo, dhi, dfield, alpha, order, V, idx);
}

void orc_spatial_op(const orc_dyn* dyn, const orc_grid* g, const double* dlo,
                    const double* dhi, const double* alpha, int order,
                    const double* V, double* L)
{
    orc_spatial_op_field(dyn, g, dlo, dhi, NULL, alpha, order, V, L);
}

/* ------------------------------------------------------------------------ */
/* Iteration                                                                 */
/* ------------------------------------------------------------------------ */

double orc_iterate_field(const orc_dyn* dyn, const orc_grid* g,
                         const double* dlo, const double* dhi,
                         const double* dfield, const double* alpha, double dt,
                         int order, const double* l, const double* V,
                         double* Vnew)
{
    int64_t N = grid_size(g);
    double* Vhat = (double*)malloc((size_t)N * sizeof(double));
    double* L = (double*)malloc((size_t)N * sizeof(double));
    /* stage 1: forward Euler */
    orc_spatial_op_field(dyn, g, dlo, dhi, dfield, alpha, order, V, L);
    for (int64_t i = 0; i < N; i++) Vhat[i] = V[i] + dt * L[i];
    /* stage 2: forward Euler from Vhat, average with V, project */
    orc_spatial_op_field(dyn, g, dlo, dhi, dfield, alpha, order, Vhat, L);
    double r = 0.0;
    for (int64_t i = 0; i < N; i++) {
        double Vtil = Vhat[i] + dt * L[i];
        double avg = 0.5 * (V[i] + Vtil);
        Vnew[i] = (l[i] < avg) ? l[i] : avg;
        double diff = fabs(Vnew[i] - V[i]);
        if (!(diff <= r)) r = diff; /* a NaN difference propagates */
    }
    free(Vhat);
    free(L);
    return r;
}

double orc_iterate(const orc_dyn* dyn, const orc_grid* g, const double* dlo,
                   const double* dhi, const double* alpha, double dt,
                   int order, const double* l, const double* V, double* Vnew)
{
    return orc_iterate_field(dyn, g, dlo, dhi, NULL, alpha, dt, order, l, V, Vnew);
}

double orc_iterate_at_field(const orc_dyn* dyn, const orc_grid* g,
                            const double* dlo, const double* dhi,
                            const double* dfield, const double* alpha,
                            double dt, int order, const double* l,
                            const double* V, int64_t idx)
{
    /* Stage 2 at idx reads Vhat on the cross-shaped 5-point stencil around
     * idx; build those Vhat values from stage 1 evaluated at each of them. */
    int D = g->ndim;
    int j[4];
    unflatten(g, idx, j);
    double Lhat = 0.0;
    {
        /* Assemble a private copy of the Vhat entries the stencil touches,
         * addressed through a tiny map from flat index to value. */
        int64_t keys[1 + 4 * 4];
        double vals[1 + 4 * 4];
        int nk = 0;
        keys[nk] = idx;
        vals[nk++] = V[idx] + dt * node_op(dyn, g, dlo, dhi, dfield, alpha, order, V, idx);
        for (int i = 0; i < D; i++) {
            int64_t s = stride_of(g, i);
            for (int o = -2; o <= 2; o++) {
                if (o == 0) continue;
                int jj = j[i] + o;
                if (jj < 0 || jj >= g->n[i]) continue;
                int64_t k = idx + (int64_t)o * s;
                keys[nk] = k;
                vals[nk++] = V[k] + dt * node_op(dyn, g, dlo, dhi, dfield, alpha, order, V, k);
            }
        }
        /* L(Vhat) at idx, with the ghost rule applied to Vhat lines. */
        double x[4], pbar[4], diss = 0.0, w[5];
        for (int i = 0; i < D; i++) {
            int64_t s = stride_of(g, i);
            int n = g->n[i];
            double line[5];
            /* Vhat at in-range positions j-2..j+2 (those exist in the map). */
            for (int k = 0; k < 5; k++) {
                int jj = j[i] - 2 + k;
                line[k] = 0.0;
                if (jj >= 0 && jj < n) {
                    int64_t key = idx + (int64_t)(jj - j[i]) * s;
                    for (int q = 0; q < nk; q++)
                        if (keys[q] == key) line[k] = vals[q];
                }
            }
            /* Ghosts from the two end nodes of the line; near an end those
             * end nodes lie inside the window. */
            for (int k = 0; k < 5; k++) {
                int jj = j[i] - 2 + k;
                if (jj >= 0 && jj < n) {
                    w[k] = line[k];
                } else if (jj < 0) {
                    double a0 = line[2 - j[i]], a1 = line[3 - j[i]];
                    w[k] = (jj == -1) ? 2.0 * a0 - a1 : 3.0 * a0 - 2.0 * a1;
                } else {
                    int e = n - 1 - j[i]; /* window offset of node n-1, minus 2 */
                    double b0 = line[2 + e], b1 = line[1 + e];
                    w[k] = (jj == n) ? 2.0 * b0 - b1 : 3.0 * b0 - 2.0 * b1;
                }
            }
            double pm, pp;
            eno_point(w, spacing(g, i), order, &pm, &pp);
            pbar[i] = 0.5 * (pp + pm);
            diss += alpha[i] * 0.5 * (pp - pm);
            x[i] = orc_coord(g, i, j[i]);
        }
        double blo[2], bhi[2];
        node_dbox(orc_num_dstb(dyn->kind), dlo, dhi, dfield, grid_size(g), idx, blo, bhi);
        Lhat = orc_hamiltonian(dyn, x, pbar, blo, bhi) + diss;
        double Vtil = vals[0] + dt * Lhat;
        double avg = 0.5 * (V[idx] + Vtil);
        return (l[idx] < avg) ? l[idx] : avg;
    }
}

double orc_iterate_at(const orc_dyn* dyn, const orc_grid* g, const double* dlo,
                      const double* dhi, const double* alpha, double dt,
                      int order, const double* l, const double* V,
                      int64_t idx)
{
    return orc_iterate_at_field(dyn, g, dlo, dhi, NULL, alpha, dt, order, l, V, idx);
}

double orc_residual_band(int64_t N, const double* V, const double* Vnew, double band)
{
    double r = 0.0;
    for (int64_t i = 0; i < N; i++) {
        if (band > 0.0 && fabs(V[i]) >= band && fabs(Vnew[i]) >= band) continue;
        double diff = fabs(Vnew[i] - V[i]);
        if (!(diff <= r)) r = diff; /* a NaN difference propagates */
    }
    return r;
}

int orc_solve_field(const orc_dyn* dyn, const orc_grid* g, const double* l,
                    const double* V0, const double* dlo, const double* dhi,
                    const double* dfield, double tol, double band, double cfl,
                    int order, int64_t max_iter, double* V_out,
                    int64_t* iterations, double* residual, double* dt_out,
                    double* alpha_out, double* res_hist, double* max_rise)
{
    if (!grid_valid(g) || orc_state_dim(dyn->kind) != g->ndim) return ORC_EINVAL;
    if (!(tol > 0.0) || !(cfl > 0.0 && cfl <= 1.0) || max_iter < 1) return ORC_EINVAL;
    if (!(band >= 0.0)) return ORC_EINVAL;
    if (order != 1 && order != 2) return ORC_EINVAL;
    int64_t N = grid_size(g);
    if (dfield) {
        /* every node's box must be an ordered pair of numbers */
        for (int c = 0; c < orc_num_dstb(dyn->kind); c++)
            for (int64_t i = 0; i < N; i++) {
                double a = dfield[(int64_t)(2 * c) * N + i];
                double b = dfield[(int64_t)(2 * c + 1) * N + i];
                if (!(a <= b) || !isfinite(a) || !isfinite(b)) return ORC_EINVAL;
            }
    } else {
        for (int c = 0; c < orc_num_dstb(dyn->kind); c++)
            if (!(dlo[c] <= dhi[c])) return ORC_EINVAL;
    }

    double alpha[4];
    orc_lf_alpha_field(dyn, g, dlo, dhi, dfield, alpha);
    double dt = orc_dt(g, alpha, cfl);
    if (alpha_out)
        for (int i = 0; i < g->ndim; i++) alpha_out[i] = alpha[i];
    if (dt_out) *dt_out = dt;

    double* V = (double*)malloc((size_t)N * sizeof(double));
    double* Vn = (double*)malloc((size_t)N * sizeof(double));
    /* Initialisation: cold start from l; warm start from min(l, V0). */
    for (int64_t i = 0; i < N; i++) {
        double v0 = V0 ? V0[i] : l[i];
        V[i] = (l[i] < v0) ? l[i] : v0;
    }
    double rise = -INFINITY;
    int status = ORC_NOT_CONVERGED;
    int64_t k;
    double r = 0.0;
    for (k = 0; k < max_iter; k++) {
        r = orc_iterate_field(dyn, g, dlo, dhi, dfield, alpha, dt, order, l, V, Vn);
        if (band > 0.0) r = orc_residual_band(N, V, Vn, band);
        if (max_rise)
            for (int64_t i = 0; i < N; i++)
                if (Vn[i] - V[i] > rise) rise = Vn[i] - V[i];
        if (res_hist) res_hist[k] = r;
        double* t = V;
        V = Vn;
        Vn = t;
        if (r < tol) {
            status = ORC_OK;
            k++;
            break;
        }
    }
    memcpy(V_out, V, (size_t)N * sizeof(double));
    *iterations = k;
    *residual = r;
    if (max_rise) *max_rise = rise;
    free(V);
    free(Vn);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Level transition (Sec. III-C) and refinement mask                         */
int orc_solve(const orc_dyn* dyn, const orc_grid* g, const double* l,
              const double* V0, const double* dlo, const double* dhi,
              double tol, double band, double cfl, int order, int64_t max_iter,
              double* V_out, int64_t* iterations, double* residual,
              double* dt_out, double* alpha_out, double* res_hist,
              double* max_rise)
{
    return orc_solve_field(dyn, g, l, V0, dlo, dhi, NULL, tol, band, cfl, order,
                           max_iter, V_out, iterations, residual, dt_out,
                           alpha_out, res_hist, max_rise);
}

/* ------------------------------------------------------------------------ */

int orc_interp(const orc_grid* src, const double* Vs, const orc_grid* dst,
               double* Vd)
{
    if (!grid_valid(src) || !grid_valid(dst) || src->ndim != dst->ndim) return ORC_EINVAL;
    int D = src->ndim;
    for (int i = 0; i < D; i++)
        if (src->lo[i] != dst->lo[i] || src->hi[i] != dst->hi[i]) return ORC_EINVAL;

    int64_t Nd = grid_size(dst);
    int jd[4];
    int64_t q[4];
    double t[4];
    int64_t sstr[4];
    for (int i = 0; i < D; i++) sstr[i] = stride_of(src, i);
    for (int64_t idx = 0; idx < Nd; idx++) {
        unflatten(dst, idx, jd);
        for (int i = 0; i < D; i++) {
            int64_t ns = src->n[i], nd = dst->n[i];
            int64_t num = (int64_t)jd[i] * (ns - 1);
            q[i] = num / (nd - 1);
            int64_t r = num % (nd - 1);
            if (q[i] == ns - 1) {
                q[i] = ns - 2;
                t[i] = 1.0;
            } else {
                t[i] = (double)r / (double)(nd - 1);
            }
        }
        double acc = 0.0;
        for (int c = 0; c < (1 << D); c++) {
            double w = 1.0;
            int64_t off = 0;
            for (int i = 0; i < D; i++) {
                int ci = (c >> (D - 1 - i)) & 1; /* first axis is the high bit */
                w = w * (ci ? t[i] : 1.0 - t[i]);
                off += (q[i] + ci) * sstr[i];
            }
            acc = acc + w * Vs[off];
        }
        Vd[idx] = acc;
    }
    return ORC_OK;
}

int64_t orc_refine_mask(const orc_grid* g, const double* V, uint8_t* mask)
{
    int D = g->ndim;
    orc_grid cells = *g;
    for (int i = 0; i < D; i++) cells.n[i] = g->n[i] - 1;
    int64_t Nc = 1;
    for (int i = 0; i < D; i++) Nc *= cells.n[i];
    int64_t str[4];
    for (int i = 0; i < D; i++) str[i] = stride_of(g, i);
    int64_t count = 0;
    int jc[4];
    for (int64_t c = 0; c < Nc; c++) {
        unflatten(&cells, c, jc);
        int any_safe = 0, any_unsafe = 0;
        for (int k = 0; k < (1 << D); k++) {
            int64_t off = 0;
            for (int i = 0; i < D; i++) off += (int64_t)(jc[i] + ((k >> i) & 1)) * str[i];
            if (V[off] >= 0.0) any_safe = 1;
            if (V[off] < 0.0) any_unsafe = 1;
        }
        mask[c] = (uint8_t)(any_safe && any_unsafe);
        count += mask[c];
    }
    return count;
}

/* ------------------------------------------------------------------------ */
/* Safety query: value, gradient and optimal safety control at a state      */
/* ------------------------------------------------------------------------ */

/* Gradient the scheme evaluates H with at node idx: per axis the mean of
 * the one-sided ENO derivatives, (p+_i + p-_i) / 2. */
static void node_pbar(const orc_grid* g, const double* V, int order, int64_t idx,
                      double* pbar)
{
    int D = g->ndim;
    int j[4];
    double w[5];
    unflatten(g, idx, j);
    for (int i = 0; i < D; i++) {
        int64_t s = stride_of(g, i);
        const double* line0 = V + (idx - (int64_t)j[i] * s);
        for (int k = 0; k < 5; k++) w[k] = line_value(line0, s, g->n[i], j[i] - 2 + k);
        double pm, pp;
        eno_point(w, spacing(g, i), order, &pm, &pp);
        pbar[i] = 0.5 * (pp + pm);
    }
}

int orc_query(const orc_dyn* dyn, const orc_grid* g, const double* V, int order,
              const double* dlo, const double* dhi, const double* x,
              double* value, double* grad, double* u_star)
{
    int D = g->ndim;
    int mu = orc_num_ctrl(dyn->kind), md = orc_num_dstb(dyn->kind);
    int j0[4];
    double t[4];
    int inside = 1;
    for (int i = 0; i < D; i++) {
        if (!(x[i] >= g->lo[i] && x[i] <= g->hi[i])) inside = 0;
    }
    if (!inside) {
        *value = NAN;
        for (int i = 0; i < D; i++) grad[i] = NAN;
        for (int k = 0; k < mu; k++) u_star[k] = NAN;
        return ORC_EINVAL;
    }
    /* the cell holding x: node j0 and fractions t along each axis */
    for (int i = 0; i < D; i++) {
        double s = (x[i] - g->lo[i]) / spacing(g, i);
        int j = (int)floor(s);
        if (j < 0) j = 0;
        if (j > g->n[i] - 2) j = g->n[i] - 2;
        j0[i] = j;
        t[i] = s - (double)j;
    }
    /* multilinear interpolation of V and of the node gradients over the
     * 2^D corners, in row-major order of the corner offsets */
    double v = 0.0, gr[4] = {0.0, 0.0, 0.0, 0.0}, pb[4];
    for (int c = 0; c < (1 << D); c++) {
        double wgt = 1.0;
        int64_t idx = 0;
        for (int i = 0; i < D; i++) {
            int o = (c >> (D - 1 - i)) & 1;
            wgt *= o ? t[i] : 1.0 - t[i];
            idx += (int64_t)(j0[i] + o) * stride_of(g, i);
        }
        v += wgt * V[idx];
        node_pbar(g, V, order, idx, pb);
        for (int i = 0; i < D; i++) gr[i] += wgt * pb[i];
    }
    *value = v;
    for (int i = 0; i < D; i++) grad[i] = gr[i];
    /* u* = a control vertex maximising min over d of grad . f(x, u, d);
     * of equal candidates the later vertex in enumeration order is kept,
     * which is the upper bound of every input that does not matter */
    double ulo[4], uhi[4], u[4], d[4], f[4];
    orc_ctrl_box(dyn, ulo, uhi);
    double best = -INFINITY;
    for (int vu = 0; vu < (1 << mu); vu++) {
        box_vertex(mu, ulo, uhi, vu, u);
        double worst = INFINITY;
        for (int vd = 0; vd < (1 << md); vd++) {
            box_vertex(md, dlo, dhi, vd, d);
            orc_dynamics(dyn, x, u, d, f);
            double sum = 0.0;
            for (int i = 0; i < D; i++) sum += gr[i] * f[i];
            if (sum < worst) worst = sum;
        }
        if (worst >= best) {
            best = worst;
            for (int k = 0; k < mu; k++) u_star[k] = u[k];
        }
    }
    return ORC_OK;
}

int orc_query_decomposed(int nsub, const orc_dyn* dyns, const orc_grid* grids,
                         const double* const* Vs, const int32_t* state_index,
                         const int32_t* control_index, const double* const* dlo,
                         const double* const* dhi, int order, const double* x,
                         double level, const double* u_perf, double* value,
                         int32_t* active, double* sub_value, double* grad,
                         double* u_star, double* u_out)
{
    int status = ORC_OK;
    double best = INFINITY;
    int arg = -1;
    for (int s = 0; s < nsub; s++) {
        int D = grids[s].ndim, m = orc_num_ctrl(dyns[s].kind);
        double xs[4], v, g[4], u[4];
        for (int a = 0; a < D; a++) xs[a] = x[state_index[4 * s + a]];
        if (orc_query(&dyns[s], &grids[s], Vs[s], order, dlo[s], dhi[s], xs, &v, g, u) != ORC_OK)
            status = ORC_EINVAL;
        sub_value[s] = v;
        for (int a = 0; a < D; a++) grad[state_index[4 * s + a]] = g[a];
        for (int k = 0; k < m; k++) {
            int c = control_index[s] + k;
            u_star[c] = u[k];
            /* each subsystem's own inputs are filtered on its own value */
            u_out[c] = (v >= level) ? u_perf[c] : u[k];
        }
        if (v < best) { /* the first subsystem attaining the minimum */
            best = v;
            arg = s;
        }
    }
    *value = status == ORC_OK ? best : NAN;
    *active = status == ORC_OK ? arg : -1;
    return status;
}

/* ------------------------------------------------------------------------ */
/* Localized updates (Sec. VI: localized warm starting)                     */
/* ------------------------------------------------------------------------ */

int64_t orc_band_mask(const orc_grid* g, const double* V, int k, uint8_t* node_mask)
{
    int D = g->ndim;
    int64_t N = grid_size(g);
    int64_t Nc = 1;
    int nc[4];
    for (int a = 0; a < D; a++) {
        nc[a] = g->n[a] - 1;
        Nc *= nc[a];
    }
    uint8_t* cells = (uint8_t*)malloc((size_t)Nc);
    orc_refine_mask(g, V, cells);
    int64_t count = 0;
    int j[4], c[4];
    for (int64_t i = 0; i < N; i++) {
        unflatten(g, i, j);
        int hit = 0;
        /* every cell c with max_a dist(j_a, [c_a, c_a + 1]) <= k */
        int lo[4], hi[4];
        for (int a = 0; a < D; a++) {
            lo[a] = j[a] - 1 - k < 0 ? 0 : j[a] - 1 - k;
            hi[a] = j[a] + k > nc[a] - 1 ? nc[a] - 1 : j[a] + k;
        }
        for (int a = 0; a < D; a++) c[a] = lo[a];
        while (!hit) {
            int64_t ci = 0;
            for (int a = 0; a < D; a++) ci = ci * nc[a] + c[a];
            if (cells[ci]) hit = 1;
            int a = D - 1;
            while (a >= 0 && c[a] == hi[a]) {
                c[a] = lo[a];
                a--;
            }
            if (a < 0) break;
            c[a]++;
        }
        node_mask[i] = (uint8_t)hit;
        count += hit;
    }
    free(cells);
    return count;
}

int orc_solve_masked(const orc_dyn* dyn, const orc_grid* g, const double* l,
                     const double* V0, const double* dlo, const double* dhi,
                     const double* dfield, const uint8_t* mask, double tol,
                     double cfl, int order, int64_t max_iter, double* V_out,
                     int64_t* iterations, double* residual)
{
    if (!grid_valid(g) || orc_state_dim(dyn->kind) != g->ndim || !mask) return ORC_EINVAL;
    if (!(tol > 0.0) || !(cfl > 0.0 && cfl <= 1.0) || max_iter < 1) return ORC_EINVAL;
    if (order != 1 && order != 2) return ORC_EINVAL;
    int64_t N = grid_size(g);
    double alpha[4];
    orc_lf_alpha_field(dyn, g, dlo, dhi, dfield, alpha);
    double dt = orc_dt(g, alpha, cfl);
    double* V = (double*)malloc((size_t)N * sizeof(double));
    double* Vhat = (double*)malloc((size_t)N * sizeof(double));
    double* Vn = (double*)malloc((size_t)N * sizeof(double));
    double* L = (double*)malloc((size_t)N * sizeof(double));
    for (int64_t i = 0; i < N; i++) {
        double v0 = V0 ? V0[i] : l[i];
        V[i] = (l[i] < v0) ? l[i] : v0;
    }
    int status = ORC_NOT_CONVERGED;
    int64_t k;
    double r = 0.0;
    for (k = 0; k < max_iter; k++) {
        /* the RK2 step of orc_iterate at the masked nodes; every other node
         * keeps its value in both stages (boundary data for the stencils) */
        orc_spatial_op_field(dyn, g, dlo, dhi, dfield, alpha, order, V, L);
        for (int64_t i = 0; i < N; i++) Vhat[i] = mask[i] ? V[i] + dt * L[i] : V[i];
        orc_spatial_op_field(dyn, g, dlo, dhi, dfield, alpha, order, Vhat, L);
        r = 0.0;
        for (int64_t i = 0; i < N; i++) {
            if (!mask[i]) {
                Vn[i] = V[i];
                continue;
            }
            double Vtil = Vhat[i] + dt * L[i];
            double avg = 0.5 * (V[i] + Vtil);
            Vn[i] = (l[i] < avg) ? l[i] : avg;
            double diff = fabs(Vn[i] - V[i]);
            if (!(diff <= r)) r = diff;
        }
        double* t = V;
        V = Vn;
        Vn = t;
        if (r < tol) {
            status = ORC_OK;
            k++;
            break;
        }
    }
    memcpy(V_out, V, (size_t)N * sizeof(double));
    *iterations = k;
    *residual = r;
    free(V);
    free(Vhat);
    free(Vn);
    free(L);
    return status;
}
