/*
 * fr_dvm.h -- C ABI of libfrdvm, the MI355X (gfx950) implementation of the
 * explicit residual-and-update step of a flux-reconstruction (FR)
 * discretisation of the Boltzmann-BGK / ES-BGK equation on hexahedra, applied
 * to every node of a conservative discrete velocity model.
 *
 * Paper: T. Dzanic & L. Martinelli, "Direct molecular gas dynamics
 * simulations of re-entry vehicles via the Boltzmann equation",
 * arXiv 2312.06567.  Section "Governing equations" defines the moments
 * (eq. moments), the BGK / ES-BGK operator and tau; Section "Numerical
 * method" defines the FR scheme (solution/flux nodes, corrected flux,
 * upwind common flux, eq. transport) and the conservative discrete velocity
 * model (eq. discrete_compatibility).
 *
 * Conventions
 *  - Layout of a distribution f: f[e][s][k], row-major, velocity index k
 *    fastest.  s = i + n (j + n l) over the (p+1)^3 Gauss-Legendre solution
 *    points of element e (x fastest), k = i + n0 (j + n1 l) over the velocity
 *    grid (x fastest).
 *  - Element types: hexahedra with 8 (trilinear) or 27 (triquadratic) nodes
 *    listed x-fastest.  Faces: face = 2 d + side, side 0 at xi_d = -1, side 1
 *    at xi_d = +1.
 *  - All f / R / S buffers are caller-owned DEVICE pointers of the handle's
 *    precision (double for FR_DVM_FP64, float for FR_DVM_FP32 and
 *    FR_DVM_FP32_DEV).  Q / Qp /
 *    totals are caller-owned DEVICE double buffers unless said otherwise.
 *    The library never frees or reallocates caller memory.
 *  - Every call is asynchronous on the handle's stream (default: the null
 *    stream) unless documented as synchronising.  Calls on one handle are not
 *    thread safe.
 *  - Return value: FR_DVM_OK (0) or a negative FR_DVM_E* code; the message is
 *    kept in fr_dvm_last_error(h).  A kernel fault surfaces at the next
 *    synchronising call.  Per-point Newton failure is not an error (see
 *    fr_dvm_newton_stats).
 */
#ifndef FR_DVM_H
#define FR_DVM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FR_DVM_OK 0
#define FR_DVM_EINVAL (-1)      /* invalid argument or inconsistent mesh */
#define FR_DVM_ENOMEM (-2)      /* device allocation failed */
#define FR_DVM_EHIP (-3)        /* HIP runtime error */
#define FR_DVM_EUNSUPPORTED (-4) /* valid input the library does not handle */
#define FR_DVM_ESCRATCH (-5)     /* request larger than the fixed scratch of a
                                    no-allocation entry point */

/* collision models (Section "Governing equations") */
#define FR_DVM_BGK 0
#define FR_DVM_ESBGK 1
#define FR_DVM_FREE 2 /* collisionless transport (S = 0), for verification */

/* storage / arithmetic precision of f and of the FR operators */
#define FR_DVM_FP64 0
#define FR_DVM_FP32 1
/* FP32 deviation storage: f buffers are float, the FR/RK arithmetic of a
 * stage is FP32, moments and Newton FP64.  Inside one fr_dvm_rk_step(s)
 * call every stage leaves its result in the caller's buffer as the FP32
 * deviation d = f - r_e from an element reference r_e, and its outflow
 * traces likewise: r_e(u) = exp of a quadratic exponent in u whose
 * coefficients are the means over the element's solution points of those
 * of the conservative equilibria the stage's Newton solve found there
 * (eq. discrete_compatibility), evaluated in FP32 (the exponent from the
 * coefficients and the velocity rounded to FP32, then the hardware exp2: an
 * FP32 number, the same bits wherever it is evaluated).  The next stage
 * reads f = r_e + d, and the exact moments of r_e are added to those of d.
 * The call's first stage reads plain f and its last stage leaves plain f,
 * rounded to FP32 (stochastically).  Within an element f stays close to one
 * reference, so the stored deviation and the arithmetic on it carry a small
 * fraction of the rounding error of FP32 f.  With FR_DVM_SSPRK3 the step's
 * initial value (read by the second and third stages) stays a deviation from
 * the references it was written with.  Periodic box meshes, monatomic gas,
 * both RK schemes, collision models BGK / ES-BGK, no positivity limiter and
 * no overlap; other calls (residual, collide,
 * moments, Kn) take f as plain float values and equal FR_DVM_FP32. */
#define FR_DVM_FP32_DEV 2

/* Newton initial guess for the conservative equilibrium */
#define FR_DVM_GUESS_COLD 0 /* continuous equilibrium of the moments of f */
#define FR_DVM_GUESS_WARM 1 /* previous solution at the same point */
#define FR_DVM_GUESS_MLP 2  /* learned guess (fr_dvm_mlp_set_weights) */
#define FR_DVM_GUESS_MLP_WARM 3 /* learned guess where no previous solution exists, warm afterwards */

/* explicit time integration (the paper names no scheme) */
#define FR_DVM_SSPRK3 0   /* three-stage SSP-RK, Shu-Osher form */
#define FR_DVM_LSRK3_2N 1 /* Williamson's three-stage low-storage scheme */

/* per-point Newton status */
#define FR_DVM_NEWTON_OK 0
#define FR_DVM_NEWTON_FALLBACK 1 /* no convergence: continuous g(Q) used */
#define FR_DVM_NEWTON_NONREAL 2  /* rho <= 0 or theta <= 0: no relaxation */
#define FR_DVM_NEWTON_ESGUARD 3  /* ES tensor near-singular: BGK used there */

typedef struct fr_dvm *fr_dvm_t; /* opaque, library-owned */

/* Mesh, caller-owned HOST arrays, copied at create. */
typedef struct {
    int32_t n_elem, n_nodes, geom_order; /* geom_order 1 (8-node) or 2 (27-node) */
    const double *nodes;                 /* [n_nodes][3] */
    const int32_t *elem_nodes;           /* [n_elem][8 | 27], x-fastest tensor order */
    const int32_t *nbr_elem;             /* [n_elem][6], -1 on a boundary face */
    const int8_t *nbr_face;              /* [n_elem][6] neighbour's face number */
    const int8_t *nbr_orient;            /* [n_elem][6] face-point map: bit0 swaps the two
                                            face indices (a,b), bit1 reverses the first,
                                            bit2 the second; (a,b) run along the two other
                                            reference axes in increasing order */
    const int8_t *bc;                    /* [n_elem][6] 0 interior/periodic, 1 farfield,
                                            2 diffuse isothermal wall, 3 specular
                                            (symmetry) wall: a plane normal to a
                                            coordinate axis, velocity grid symmetric
                                            in that axis */
} fr_dvm_mesh;

/* Uniform Cartesian velocity grid, closed (end points are nodes), trapezoid
 * weights (Section "Numerical method": Cartesian velocity nodes, strictly
 * positive integration operator M).  An axis with n = 1 has one node at umin
 * with weight 1. */
typedef struct {
    int32_t n[3];
    double umin[3], umax[3];
} fr_dvm_vgrid;

typedef struct {
    int32_t model;        /* FR_DVM_BGK | FR_DVM_ESBGK | FR_DVM_FREE */
    double prandtl;       /* ES-BGK Prandtl number (ignored for BGK) */
    double mu_ref, theta_ref, omega; /* power law mu = mu_ref (theta/theta_ref)^omega */
    int32_t visc_law;     /* 0 power law, 1 Sutherland with theta_s */
    double theta_s;
    int32_t precision;    /* FR_DVM_FP64 | FR_DVM_FP32 | FR_DVM_FP32_DEV */
    double newton_tol;    /* max-norm of the scaled compatibility residual */
    int32_t newton_max_iter;
    int32_t guess;        /* FR_DVM_GUESS_* */
    int32_t rk;           /* FR_DVM_SSPRK3 | FR_DVM_LSRK3_2N */
    double farfield[5];   /* rho, Ux, Uy, Uz, theta of the farfield Maxwellian (bc 1) */
    double theta_wall;    /* diffuse wall temperature (bc 2), wall at rest */
    int32_t overlap;      /* rk_step(s): 1 = the Newton solve of the next stage runs
                             on a second library-owned stream, half of the elements
                             at a time, while the current stage still streams the
                             other half; 0 = one stream, stage and Newton in turn.
                             Results are identical.  Box path only: ignored on
                             general meshes. */
    int32_t positivity;   /* 1: positivity limiter on every RK stage value (the
                             cited positivity-preserving FR scheme of Section
                             "Numerical method"): per element and state value,
                             the polynomial is scaled about its element mean
                             (Gauss weights x |J|) so that it is nonnegative at
                             the solution and flux points; element integrals,
                             hence all moments, are kept.  Runs in the
                             general-mesh stage kernel: a periodic box handle
                             moves to that path for good at the first
                             fr_dvm_set_params with positivity 1.  0: off. */
} fr_dvm_params;

/* Fill p with defaults: BGK, Pr 1, mu_ref 1e-3, theta_ref 1, omega 0.81,
 * FP64, tol 1e-13, 50 iterations, cold guess, SSP-RK3, overlap 0,
 * positivity 0. */
void fr_dvm_default_params(fr_dvm_params *p);

/* Create a handle for a mesh, FR order p (solution points (p+1)^3 per
 * element) and velocity grid.  Builds the FR operators, metrics,
 * connectivity and velocity tables on the device of the current HIP device.
 * Periodic boxes of axis-aligned hexahedra (every face on the opposite face
 * of its neighbour, orientation 0) take the fused box path; any other mesh
 * (27-node curved elements, any orientation codes, farfield / wall faces)
 * the general path with pointwise metrics and full traces.  A face pair must
 * conform: at matched flux points opposite normals, positions differing by
 * one vector (zero, or a period).  Returns FR_DVM_EINVAL for an inconsistent
 * mesh (non-positive Jacobian, non-conforming or asymmetric neighbours, a
 * boundary face without tag 1, 2 or 3, a specular face that is not a
 * coordinate plane), FR_DVM_EUNSUPPORTED for p outside 1..3. */
int fr_dvm_create(const fr_dvm_mesh *mesh, int order, const fr_dvm_vgrid *grid, fr_dvm_t *out);

/* fr_dvm_create with a choice of solution points per axis (Section
 * "Implementation & problem setup": the paper places Gauss-Lobatto points on
 * tensor-product elements): nodes FR_DVM_NODES_GAUSS (Gauss-Legendre, what fr_dvm_create
 * uses) or FR_DVM_NODES_LOBATTO (Gauss-Lobatto, order >= 1; points on the
 * element faces).  The correction functions recover nodal DG with the exact
 * mass matrix in both cases; moments' domain totals use the same rule's
 * weights.  FR_DVM_EINVAL for another value. */
#define FR_DVM_NODES_GAUSS 0
#define FR_DVM_NODES_LOBATTO 1
int fr_dvm_create_nodes(const fr_dvm_mesh *mesh, int order, int nodes, const fr_dvm_vgrid *grid,
                        fr_dvm_t *out);

/* fr_dvm_create_nodes for a gas with delta >= 0 internal degrees of freedom
 * (Section "Governing equations", the reduced distribution pair).  delta > 0:
 * the state is the pair (F, G), every state buffer (f, R, S, the RK
 * register) holds per solution point F then G, nu values each
 * ([e][s][2][k]); F and G are advected alike and relax with the same tau to
 * g and delta theta / 2 g; theta follows from E - rho |U|^2 / 2 =
 * (3 + delta)/2 rho theta with E the translational energy of F plus the
 * integral of G; moments report that total E.  Walls emit delta theta_w / 2
 * times their F state as G, the farfield G is delta theta_inf / 2 times the
 * farfield F.  Periodic axis-aligned boxes keep the fused box path (F's
 * chunks, then G's, per element), other meshes the general path; the
 * learned Newton start is replaced by the cold start.  delta = 0 is
 * fr_dvm_create_nodes.
 * FR_DVM_EINVAL for delta < 0 or not finite. */
int fr_dvm_create_gas(const fr_dvm_mesh *mesh, int order, int nodes, double delta,
                      const fr_dvm_vgrid *grid, fr_dvm_t *out);

/* Mixed meshes of straight hexahedra, prisms and tetrahedra (Section
 * "Implementation & problem setup": the paper's meshes mix prisms and
 * tetrahedra, with alpha-optimised solution points on simplices and
 * Gauss-Lobatto points on tensor-product elements).
 *
 * Element types and their vertex order (elem_nodes, the type's vertices
 * first, the rest of the 8 slots ignored):
 *   FR_DVM_HEX   8 vertices, x-fastest over the reference cube [-1,1]^3;
 *   FR_DVM_PRISM 6 vertices: the triangle v0 v1 v2 at reference zeta = -1
 *                (reference triangle (-1,-1), (1,-1), (-1,1)) and v3 v4 v5
 *                over it at zeta = +1;
 *   FR_DVM_TET   4 vertices: reference (-1,-1,-1), (1,-1,-1), (-1,1,-1),
 *                (-1,-1,1).
 * Every element must be the affine image of its reference element with a
 * positive Jacobian (straight elements, parallelogram quadrilateral faces).
 * Faces (nbr_elem / nbr_face numbering), by their vertices:
 *   hexahedron 0:{0,2,4,6} 1:{1,3,5,7} 2:{0,1,4,5} 3:{2,3,6,7} 4:{0,1,2,3} 5:{4,5,6,7};
 *   prism      0:{0,1,2} 1:{3,4,5} 2:{0,1,4,3} 3:{1,2,5,4} 4:{2,0,3,5};
 *   tetrahedron 0:{0,1,2} 1:{0,1,3} 2:{1,2,3} 3:{0,2,3}.
 * Every face must have a neighbour (closed or periodic meshes); the face
 * points of two neighbours are matched by position, modulo the period.
 *
 * Solution points (order p = 1..3), element after element in the state
 * buffers ([point][velocity]): hexahedron the Gauss-Lobatto tensor points
 * i + n (j + n l); prism the triangle points t + n_tri l over the
 * Gauss-Lobatto points l of zeta; triangle and tetrahedron the alpha-
 * optimised warp & blend points, which for p <= 3 are the vertices, the
 * Gauss-Lobatto points along every edge and the face centroids (tetrahedron
 * p = 3), indexed by barycentric (i, j[, k]) / p with i + j [+ k] <= p, the
 * last index outermost.  The flux points of a face are the solution points
 * on it.  The scheme is FR with the DG-recovering correction (nodal DG with
 * exact mass matrices) and the upwind flux.
 *
 * The handle treats every solution point as an element of one point:
 * fr_dvm_sizes reports n_elem = the number of points and ns = 1, and
 * residual / collide / moments / rk_step(s) / dt / newton_* work on
 * [points][nu] buffers; the domain totals weight each point by the
 * integral of its basis function.  dt uses h = element volume / largest
 * face area.  FP64 and FP32, BGK / ES-BGK / free, both RK schemes; no
 * FR_DVM_FP32_DEV, no positivity limiter, no reduced pair, no
 * fr_dvm_kn_gll (FR_DVM_EUNSUPPORTED). */
#define FR_DVM_HEX 0
#define FR_DVM_PRISM 1
#define FR_DVM_TET 2
typedef struct {
    int32_t n_elem, n_nodes;
    const double *nodes;       /* [n_nodes][3] */
    const int8_t *elem_type;   /* [n_elem] FR_DVM_HEX | FR_DVM_PRISM | FR_DVM_TET */
    const int32_t *elem_nodes; /* [n_elem][8] */
    const int32_t *nbr_elem;   /* [n_elem][6] neighbour across each face (slots past the type's faces ignored) */
    const int8_t *nbr_face;    /* [n_elem][6] that neighbour's face */
    double period[3];          /* translation of the periodic domain along x, y, z (0: none) */
} fr_dvm_mixed_mesh;
int fr_dvm_create_mixed(const fr_dvm_mixed_mesh *mesh, int order, const fr_dvm_vgrid *grid, fr_dvm_t *out);

/* Set physics / precision / solver parameters; allocates the work buffers
 * of the chosen precision.  Must be called before any compute call. */
int fr_dvm_set_params(fr_dvm_t h, const fr_dvm_params *p);

/* Run subsequent calls on this hipStream_t (passed as void*). */
int fr_dvm_set_stream(fr_dvm_t h, void *stream);

/* Sizes and the bytes of device memory the handle owns.  nu counts velocity
 * nodes; a state of the reduced pair (fr_dvm_create_gas, delta > 0) holds
 * 2 nu values per solution point. */
int fr_dvm_sizes(fr_dvm_t h, int64_t *n_elem, int32_t *ns, int32_t *nf, int32_t *nu,
                 size_t *workspace_bytes);

/* Host copies of the velocity nodes [nu][3] and weights [nu] (either may be NULL). */
int fr_dvm_velocity_nodes(fr_dvm_t h, double *u, double *w);

/* Explicit time step dt = cfl h_min / ((2p+1) max_k sum_d |u_k,d|), h = 2|J|/|a^d|. */
int fr_dvm_dt(fr_dvm_t h, double cfl, double *dt);

/* Advective FR residual R = -div(u f) at every solution point and velocity
 * node (eq. transport with the corrected flux and the upwind interface
 * flux; boundary exteriors from bc tags).  f, R: device [e][s][k]. */
int fr_dvm_residual(fr_dvm_t h, const void *f, void *R);

/* Collision source S = (g(Q') - f)/tau, where g(Q') is the conservative
 * equilibrium with the same discrete moments as f (eq.
 * discrete_compatibility), solved per point by FP64 Newton.  If accumulate,
 * S += source.  Qp (nullable, device double [e][s][5]) receives the
 * primitive state (rho', U', theta') of g(Q').  f, S: device [e][s][k]. */
int fr_dvm_collide(fr_dvm_t h, const void *f, void *S, double *Qp, int accumulate);

/* Discrete moments Q = M.(f psi), psi = (1, u, |u|^2/2) (eq. moments) into
 * device Q[e][s][5]; totals (nullable, HOST double[5]) receives the domain
 * integrals (Gauss weights x |J|).  Synchronises when totals != NULL. */
int fr_dvm_moments(fr_dvm_t h, const void *f, double *Q, double *totals);

/* Gradient-length local Knudsen number at every solution point (Section
 * "Results", the continuum-breakdown parameter): Kn = lambda |grad rho| / rho,
 * lambda = mu(theta)/rho sqrt(pi / (2 theta)) with the handle's viscosity law,
 * grad rho the derivative of the element's solution polynomial of the
 * discrete density.  f: device [e][s][k] in the handle's precision; kn:
 * device double [e][s], 0 where rho <= 0 or theta <= 0.  Asynchronous on the
 * handle's stream; overwrites the handle's moment buffer. */
int fr_dvm_kn_gll(fr_dvm_t h, const void *f, double *kn);

/* Advance f (device, in place) by one / nsteps explicit steps of size dt of
 * df/dt = R(f) + S(f) with the scheme chosen in the parameters. */
int fr_dvm_rk_step(fr_dvm_t h, void *f, double dt);
int fr_dvm_rk_steps(fr_dvm_t h, void *f, double dt, int nsteps);

/* Newton statistics accumulated since the last reset (synchronising):
 * iters_hist[64] histogram of iterations (linear solves) per point solve,
 * number of fallback and ES-guard points, total residual evaluations (passes
 * over the velocity grid), and the largest final scaled residual.  Any
 * pointer may be NULL.  reset != 0 clears the counters afterwards. */
int fr_dvm_newton_stats(fr_dvm_t h, int64_t *iters_hist, int64_t *n_fallback,
                        int64_t *n_guard, int64_t *n_evals, double *max_resid, int reset);

/* Per-point outcome of the handle's most recent conservative-equilibrium
 * solve (the last Newton launch of rk_step(s), or collide): status
 * (FR_DVM_NEWTON_*), linear solves and final scaled residual of every
 * solution point, into caller-owned DEVICE arrays int32 status[e][s], int32
 * iters[e][s], double resid[e][s] (any may be NULL).  Asynchronous on the
 * handle's stream.  FR_DVM_EINVAL before the first solve. */
int fr_dvm_newton_points(fr_dvm_t h, int32_t *status, int32_t *iters, double *resid);

/* Weights of the learned Newton initial guess: an MLP 7 -> H -> H -> H -> 5
 * with SiLU activations (FP32, layout documented in fr_dvm_mlp.h).  n is the
 * number of floats; the guess mode FR_DVM_GUESS_MLP uses them. */
int fr_dvm_mlp_set_weights(fr_dvm_t h, const float *w, size_t n);

/* Kernel timing with HIP events recorded on the handle's stream around each
 * launch.  fr_dvm_profile(h, 1) starts recording (0 stops);
 * fr_dvm_profile_read (synchronising) returns, per kernel kind, the summed
 * milliseconds and launch counts: [0] fused FR stage, [1] Newton, [2] prime
 * (traces/moments of the incoming f), [3] other.  reset != 0 clears them. */
#define FR_DVM_PROF_KINDS 4
int fr_dvm_profile(fr_dvm_t h, int enable);
int fr_dvm_profile_read(fr_dvm_t h, double *ms, int64_t *launches, int reset);

/* HBM bandwidth probe (no handle): plain copy of nbytes from src to dst,
 * both device pointers, 16-byte loads and stores, on stream (hipStream_t as
 * void*, may be NULL).  nbytes must be a multiple of 16 and the ranges must
 * not overlap.  Used to calibrate hardware byte counters against a kernel
 * of known traffic. */
int fr_dvm_hbm_copy(void *dst, const void *src, size_t nbytes, void *stream);

const char *fr_dvm_last_error(fr_dvm_t h);
void fr_dvm_destroy(fr_dvm_t h);

#ifdef __cplusplus
}
#endif
#endif /* FR_DVM_H */
