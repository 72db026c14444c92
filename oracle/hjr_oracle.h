/*
 * hjr_oracle.h -- plain, single-threaded FP64 reference for the grid-based
 * Hamilton-Jacobi reachability safe-set solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this code; only the test-suite, the smoke check and the CPU
 * baseline of the benchmark load it.  It shares no header, helper, table or
 * constant with the HIP path.
 *
 * Sign convention.  The paper (Sec. II-A, eq. (1)-(2)) uses a cost c <= 0
 * inside the constraint set, V = sup_d inf_u max_tau c(xi(tau)), projection
 * max{c - V, .} and Hamiltonian min_u max_d <grad V, f>.  This code uses the
 * negated quantities l = -c, V = -V_paper, so
 *     0 = min{ l - V , D_tau V + max_u min_d <grad V, f> },
 * the projection is V <- min(l, V), and the safe set is { V* >= 0 }.
 *
 * Discretisation (the paper does not name one): second-order ENO upwind
 * derivatives (Osher & Shu 1991; Osher & Fedkiw, "Level Set Methods", ch. 3),
 * global Lax-Friedrichs dissipation (Crandall-Lions / Osher-Shu), and the
 * two-stage TVD Runge-Kutta step of Shu & Osher (1988), CFL number 0.8.
 *
 * All arrays are dense, row-major, last dimension fastest.
 */
#ifndef HJR_ORACLE_H
#define HJR_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_QUAD_Z2D = 0, ORC_QUAD_X4D = 1, ORC_DI2X2 = 2, ORC_QUAD_X4DV = 3 };

enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_NOT_CONVERGED = 3 };

typedef struct orc_grid {
    int32_t ndim;
    int32_t n[4];
    double lo[4];
    double hi[4];
} orc_grid;

/* Dynamics.  Parameters per kind:
 *   ORC_QUAD_Z2D  state (z, vz):  p = {k, g, u_lo, u_hi}
 *                 f = (vz, k*u - g + d),  u in [u_lo, u_hi], d channel 0.
 *   ORC_QUAD_X4D  state (x, vx, theta, omega):  p = {g, d1, d0, n0, s_max}
 *                 f = (vx + d, g*tan(theta), -d1*theta + omega, -d0*theta + n0*S)
 *                 S in [-s_max, s_max], d channel 0.
 *   ORC_QUAD_X4DV the x-subsystem as the 10-D model of Sec. IV writes it,
 *                 with the disturbance on the velocity rate:
 *                 p = {g, d1, d0, n0, s_max}
 *                 f = (vx, g*tan(theta) + d, -d1*theta + omega, -d0*theta + n0*S)
 *                 S in [-s_max, s_max], d channel 0.
 *   ORC_DI2X2     two QUAD_Z2D copies "a" and "b" on a 4-D grid:
 *                 p = {k_a, g_a, ulo_a, uhi_a, k_b, g_b, ulo_b, uhi_b,
 *                      axis(z_a), axis(v_a), axis(z_b), axis(v_b)}
 *                 (axes stored as doubles), d channel 0 acts on a, 1 on b.
 */
typedef struct orc_dyn {
    int32_t kind;
    int32_t pad_;
    double p[16];
} orc_dyn;

/* Number of state dimensions / control inputs / disturbance channels. */
int orc_state_dim(int kind);
int orc_num_ctrl(int kind);
int orc_num_dstb(int kind);

/* f(x, u, d) written out component by component. */
void orc_dynamics(const orc_dyn* dyn, const double* x, const double* u,
                  const double* d, double* f);

/* Control / disturbance box vertices: ctrl_lo/ctrl_hi per input. */
void orc_ctrl_box(const orc_dyn* dyn, double* lo, double* hi);

/* H(x, p) = max over u in U of min over d in D of p . f(x, u, d), by
 * enumerating the vertices of the control and disturbance boxes (f is
 * affine in u and in d, so the extrema sit on vertices). */
double orc_hamiltonian(const orc_dyn* dyn, const double* x, const double* p,
                       const double* dlo, const double* dhi);

/* Node coordinate x_i[j] = lo_i + j * (hi_i - lo_i) / (n_i - 1). */
double orc_coord(const orc_grid* g, int axis, int j);

/* Global Lax-Friedrichs bounds: alpha_i = max over nodes and over the
 * vertices of the control and disturbance boxes of |f_i|. */
void orc_lf_alpha(const orc_dyn* dyn, const orc_grid* g, const double* dlo,
                  const double* dhi, double* alpha);

/* dt = cfl / sum_i alpha_i / dx_i. */
double orc_dt(const orc_grid* g, const double* alpha, double cfl);

/* One-sided derivatives along a single line of n samples (n >= 3), with two
 * linear-extrapolation ghost nodes on each side.  order 2 = ENO2, 1 = first
 * order.  pm[j] = D^- at j, pp[j] = D^+ at j. */
void orc_line_derivs(const double* v, int n, double h, int order, double* pm,
                     double* pp);

/* Spatial operator L(V) = H(x, (p+ + p-)/2) + sum_i alpha_i (p+_i - p-_i)/2
 * at every node. */
void orc_spatial_op(const orc_dyn* dyn, const orc_grid* g, const double* dlo,
                    const double* dhi, const double* alpha, int order,
                    const double* V, double* L);

/* One full iteration: Vhat = V + dt L(V); Vtil = Vhat + dt L(Vhat);
 * Vnew = min(l, (V + Vtil)/2).  Returns max |Vnew - V|.  Vnew may not alias V. */
double orc_iterate(const orc_dyn* dyn, const orc_grid* g, const double* dlo,
                   const double* dhi, const double* alpha, double dt,
                   int order, const double* l, const double* V, double* Vnew);

/* The same iteration evaluated at one node only (flat index idx), from the
 * full array V.  Used to check a device result at sampled nodes of a grid too
 * large to iterate here. */
double orc_iterate_at(const orc_dyn* dyn, const orc_grid* g, const double* dlo,
                      const double* dhi, const double* alpha, double dt,
                      int order, const double* l, const double* V,
                      int64_t idx);

/* Residual of one iteration, max |Vnew - V|, over the nodes near the zero
 * level set: node i is left out only if both |V[i]| >= band and
 * |Vnew[i]| >= band.  band == 0 counts every node.  A NaN value is always
 * counted, and a NaN difference makes the result NaN.  (A narrow-band stop
 * rule: the safe set { V >= 0 } depends on the values near V = 0 only.) */
double orc_residual_band(int64_t N, const double* V, const double* Vnew, double band);

/* Time-marched solve of the variational inequality until the residual of an
 * iteration (orc_residual_band with the given band; 0 = all nodes) < tol.
 *   V0 == NULL: cold start V0 = l.  Otherwise V <- min(l, V0) (warm start).
 *   res_hist (nullable, length max_iter): residual of every iteration.
 *   max_rise (nullable): max over iterations and nodes of V_{k+1} - V_k.
 * Returns ORC_OK, ORC_NOT_CONVERGED (outputs hold the last iterate) or
 * ORC_EINVAL. */
int orc_solve(const orc_dyn* dyn, const orc_grid* g, const double* l,
              const double* V0, const double* dlo, const double* dhi,
              double tol, double band, double cfl, int order, int64_t max_iter,
              double* V_out, int64_t* iterations, double* residual,
              double* dt_out, double* alpha_out, double* res_hist,
              double* max_rise);

/* Multilinear interpolation between two grids over the same box, with
 * integer index arithmetic and FP64 weights; corners summed in row-major
 * order of their offsets.  Returns ORC_EINVAL if the boxes differ. */
int orc_interp(const orc_grid* src, const double* Vs, const orc_grid* dst,
               double* Vd);

/* Refinement mask: cell c in [0, n-2]^D is 1 iff one of its 2^D corner nodes
 * has V >= 0 and another has V < 0.  Returns the number of marked cells. */
int64_t orc_refine_mask(const orc_grid* g, const double* V, uint8_t* mask);


/* ------------------------------------------------------------------------ */
/* State-dependent disturbance bounds (Sec. II-A: d in D(x); Sec. II-C: the  */
/* learned bound is a confidence interval at each state).  dfield holds, for */
/* each disturbance channel c, the lower bounds of every node at            */
/* dfield[(2c) N ...] and the upper bounds at dfield[(2c + 1) N ...] (N      */
/* nodes, row-major).  Where these functions take dlo/dhi as well, those    */
/* are used only when dfield is NULL (then they equal the constant-box      */
/* functions above).                                                        */
/* ------------------------------------------------------------------------ */

/* alpha_i = max over nodes x and over the vertices of U x D(x) of |f_i|. */
void orc_lf_alpha_field(const orc_dyn* dyn, const orc_grid* g,
                        const double* dlo, const double* dhi,
                        const double* dfield, double* alpha);

/* L(V) with the Hamiltonian of node x taken over D(x). */
void orc_spatial_op_field(const orc_dyn* dyn, const orc_grid* g,
                          const double* dlo, const double* dhi,
                          const double* dfield, const double* alpha, int order,
                          const double* V, double* L);

double orc_iterate_field(const orc_dyn* dyn, const orc_grid* g,
                         const double* dlo, const double* dhi,
                         const double* dfield, const double* alpha, double dt,
                         int order, const double* l, const double* V,
                         double* Vnew);

double orc_iterate_at_field(const orc_dyn* dyn, const orc_grid* g,
                            const double* dlo, const double* dhi,
                            const double* dfield, const double* alpha,
                            double dt, int order, const double* l,
                            const double* V, int64_t idx);

/* orc_solve with per-node bounds; ORC_EINVAL if a node's pair is not two
 * finite numbers with lower <= upper. */
int orc_solve_field(const orc_dyn* dyn, const orc_grid* g, const double* l,
                    const double* V0, const double* dlo, const double* dhi,
                    const double* dfield, double tol, double band, double cfl,
                    int order, int64_t max_iter, double* V_out,
                    int64_t* iterations, double* residual, double* dt_out,
                    double* alpha_out, double* res_hist, double* max_rise);

/* Safety query at the state x (Sec. II-A: the gradient of the converged
 * value gives the optimal safety control, the optimiser of the
 * Hamiltonian).  value: multilinear interpolation of V at x (corner
 * weights products of t and 1 - t, t the fraction of x in its cell, corners
 * summed in row-major order of their offsets); grad: the same interpolation
 * of the node gradients (p+_i + p-_i)/2 of the scheme (order 2 = ENO2);
 * u_star: a vertex of the control box maximising min over the disturbance
 * box [dlo, dhi] of grad . f(x, u, d), by enumeration; among equal vertices
 * the upper bound of an input is taken.  Returns ORC_OK, or ORC_EINVAL with
 * NaN outputs when x lies outside the grid box. */
int orc_query(const orc_dyn* dyn, const orc_grid* g, const double* V, int order,
              const double* dlo, const double* dhi, const double* x,
              double* value, double* grad, double* u_star);

/* Decomposed query (Sec. III-A: a system decoupled into subsystems has the
 * product of their safe sets, so its value is the minimum of theirs, and
 * each subsystem's safety controller drives its own inputs).  Subsystem s
 * has model dyns[s], grid grids[s], value Vs[s] and disturbance box dlo[s],
 * dhi[s]; its axis a is component state_index[4 s + a] of the full state x,
 * its controls start at control_index[s] of the full control vector.
 * Outputs: sub_value[s] (orc_query of each subsystem at its part of x),
 * value = the minimum, active = the first subsystem attaining it, grad and
 * u_star scattered to the full state / control vectors, and u_out: per
 * subsystem, its inputs from u_perf where its own value >= level, else its
 * u_star.  Returns ORC_EINVAL (value NaN, active -1) if any part of x lies
 * outside its subsystem's grid box. */
int orc_query_decomposed(int nsub, const orc_dyn* dyns, const orc_grid* grids,
                         const double* const* Vs, const int32_t* state_index,
                         const int32_t* control_index, const double* const* dlo,
                         const double* const* dhi, int order, const double* x,
                         double level, const double* u_perf, double* value,
                         int32_t* active, double* sub_value, double* grad,
                         double* u_star, double* u_out);

/* Localized update (Sec. VI names localized warm starting as a further
 * speed-up).  Band of a warm start: node i is in it iff some cell straddling
 * the zero level set of V (orc_refine_mask) lies within k cells of it: for
 * every axis, the cell's index range [c_a, c_a + 1] is at most k nodes from
 * i_a.  Writes node_mask (N bytes) and returns its number of ones. */
int64_t orc_band_mask(const orc_grid* g, const double* V, int k, uint8_t* node_mask);

/* orc_solve_field restricted to the nodes with mask[i] != 0: both RK stages
 * and the projection update those nodes only; every other node keeps its
 * initial value min(l, V0) throughout and serves as boundary data; the
 * residual runs over the masked nodes (0 if there are none, so the first
 * step stops).  LF bounds and dt over the whole grid as in orc_solve. */
int orc_solve_masked(const orc_dyn* dyn, const orc_grid* g, const double* l,
                     const double* V0, const double* dlo, const double* dhi,
                     const double* dfield, const uint8_t* mask, double tol,
                     double cfl, int order, int64_t max_iter, double* V_out,
                     int64_t* iterations, double* residual);

#ifdef __cplusplus
}
#endif

#endif
