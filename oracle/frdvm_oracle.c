/*
 * frdvm_oracle.c -- plain FP64 CPU oracle of the flux-reconstruction x
 * conservative discrete-velocity Boltzmann-BGK/ES-BGK step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the HIP library.
 *
 * Reference: Dzanic & Martinelli, "Direct molecular gas dynamics simulations
 * of re-entry vehicles via the Boltzmann equation" (arXiv 2312.06567).
 * Every function names the passage it follows.  Velocity-space sums are
 * accumulated in long double; everything stored is double.
 *
 * Readings of passages the paper leaves open (also listed in the design notes):
 *  - monatomic gas (no internal energy, delta = 0, gamma = 5/3);
 *  - velocity grid closed (end points included), trapezoid weights;
 *  - Gauss-Legendre solution points on hexahedra, Huynh's g_DG correction;
 *  - conservative equilibrium parameterised as an exponential of a quadratic
 *    in u (Mieussens form); for ES-BGK the quadratic's shape is fixed by the
 *    continuous ES temperature tensor and only its scale is solved for;
 *  - Newton in the frame shifted by U and scaled by sqrt(theta), backtracking
 *    on the residual 2-norm (step halved per rejected trial, at most 40
 *    rejected trials per solve), stop at max-norm <= tol, then one extra step.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef long double ld;

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2

/* Newton status codes per solution point */
#define ORC_NEWTON_OK 0
#define ORC_NEWTON_FALLBACK 1 /* no convergence: continuous equilibrium g(Q) used */
#define ORC_NEWTON_NONREAL 2  /* rho <= 0 or theta <= 0: no relaxation */
#define ORC_NEWTON_ESGUARD 3  /* ES temperature tensor near-singular: BGK used */

/* ------------------------------------------------------------------------ */
/* 1D polynomial tools (Section "Numerical method": nodal basis, correction) */
/* ------------------------------------------------------------------------ */

/* Legendre P_n(x) and P_n'(x) by the three-term (Bonnet) recurrence. */
static void legendre(int n, ld x, ld *P, ld *dP) {
    ld p0 = 1.0L, p1 = x, d0 = 0.0L, d1 = 1.0L;
    if (n == 0) { *P = 1.0L; *dP = 0.0L; return; }
    for (int k = 1; k < n; ++k) {
        ld p2 = ((2 * k + 1) * x * p1 - k * p0) / (k + 1);
        ld d2 = d0 + (2 * k + 1) * p1; /* P'_{k+1} = P'_{k-1} + (2k+1) P_k */
        p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    }
    *P = p1; *dP = d1;
}

/* n Gauss-Legendre nodes (ascending) and weights on [-1,1]. */
int orc_gauss_legendre(int n, double *xi, double *wq) {
    if (n < 1 || n > 32) return ORC_EINVAL;
    for (int i = 0; i < n; ++i) {
        ld x = -cosl(3.14159265358979323846264338327950288L * (i + 0.75L) / (n + 0.5L));
        ld P, dP;
        for (int it = 0; it < 100; ++it) {
            legendre(n, x, &P, &dP);
            ld dx = P / dP;
            x -= dx;
            if (fabsl(dx) < 1e-19L) break;
        }
        legendre(n, x, &P, &dP);
        xi[i] = (double)x;
        if (wq) wq[i] = (double)(2.0L / ((1.0L - x * x) * dP * dP));
    }
    return ORC_OK;
}

/* n >= 2 Gauss-Lobatto-Legendre nodes (ascending: -1, the roots of
 * P'_{n-1}, +1) and weights 2 / (n (n-1) P_{n-1}(x)^2) on [-1,1]. */
int orc_gauss_lobatto(int n, double *xi, double *wq) {
    if (n < 2 || n > 32) return ORC_EINVAL;
    int p = n - 1;
    for (int i = 0; i < n; ++i) {
        ld x = -cosl(3.14159265358979323846264338327950288L * i / p);
        if (i > 0 && i < p) {
            /* Newton on P_p'(x), with P_p'' from the Legendre equation */
            for (int it = 0; it < 100; ++it) {
                ld P, dP;
                legendre(p, x, &P, &dP);
                ld d2P = (2.0L * x * dP - p * (p + 1.0L) * P) / (1.0L - x * x);
                ld dx = dP / d2P;
                x -= dx;
                if (fabsl(dx) < 1e-19L) break;
            }
        }
        ld P, dP;
        legendre(p, x, &P, &dP);
        xi[i] = (double)x;
        if (wq) wq[i] = (double)(2.0L / (p * (p + 1.0L) * P * P));
    }
    return ORC_OK;
}

/* Solution points of one axis: set 0 Gauss-Legendre, set 1 Gauss-Lobatto. */
static int solution_points(int set, int n, double *xi, double *wq) {
    return set == 1 ? orc_gauss_lobatto(n, xi, wq) : orc_gauss_legendre(n, xi, wq);
}

/* Lagrange basis l_j(x) on nodes z[0..n-1]. */
static ld lagr(int n, const ld *z, int j, ld x) {
    ld v = 1.0L;
    for (int m = 0; m < n; ++m)
        if (m != j) v *= (x - z[m]) / (z[j] - z[m]);
    return v;
}

/* Derivative l_j'(x): sum over the dropped factor (product rule). */
static ld lagr_d(int n, const ld *z, int j, ld x) {
    ld s = 0.0L;
    for (int r = 0; r < n; ++r) {
        if (r == j) continue;
        ld t = 1.0L / (z[j] - z[r]);
        for (int m = 0; m < n; ++m)
            if (m != j && m != r) t *= (x - z[m]) / (z[j] - z[m]);
        s += t;
    }
    return s;
}

/*
 * One-dimensional FR operators for degree p on Gauss-Legendre (set 0) or
 * Gauss-Lobatto (set 1) points
 * (Section "Numerical method", the corrected flux and its correction
 * functions h_i chosen to recover nodal DG).
 *   xi[n]       solution points, n = p+1
 *   D[n*n]      D[i*n+j] = l_j'(xi_i)
 *   lamL/lamR   l_j(-1), l_j(+1)            (trace to the two faces)
 *   cM/cP       -gL'(xi_i), +gR'(xi_i)      (correction at the -1 and +1 face)
 * with the DG correction functions (right/left Radau polynomials)
 *   gL(x) = (-1)^n/2 (P_n - P_{n-1}),  gR(x) = 1/2 (P_n + P_{n-1}).
 */
int orc_fr_ops_set(int p, int set, double *xi, double *D, double *lamL, double *lamR,
                   double *cM, double *cP) {
    int n = p + 1;
    if (p < 0 || p > 8 || (set == 1 && p < 1)) return ORC_EINVAL;
    double xd[16];
    ld z[16];
    solution_points(set, n, xd, NULL);
    for (int i = 0; i < n; ++i) { z[i] = xd[i]; xi[i] = xd[i]; }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            D[i * n + j] = (double)lagr_d(n, z, j, z[i]);
    for (int j = 0; j < n; ++j) {
        lamL[j] = (double)lagr(n, z, j, -1.0L);
        lamR[j] = (double)lagr(n, z, j, 1.0L);
    }
    ld sgn = (n % 2 == 0) ? 1.0L : -1.0L;
    for (int i = 0; i < n; ++i) {
        ld Pn, dPn, Pm, dPm;
        legendre(n, z[i], &Pn, &dPn);
        legendre(n - 1, z[i], &Pm, &dPm);
        ld dgL = sgn * 0.5L * (dPn - dPm);
        ld dgR = 0.5L * (dPn + dPm);
        cM[i] = (double)(-dgL);
        cP[i] = (double)dgR;
    }
    return ORC_OK;
}

int orc_fr_ops(int p, double *xi, double *D, double *lamL, double *lamR, double *cM, double *cP) {
    return orc_fr_ops_set(p, 0, xi, D, lamL, lamR, cM, cP);
}

/* ------------------------------------------------------------------------ */
/* Geometry of hexahedral elements                                           */
/* ------------------------------------------------------------------------ */

static inline int sidx(int n, int i, int j, int l) { return i + n * (j + n * l); }

/* Solution-point index of the m-th point, along axis d, of the line through
 * face point (a,b); (a,b) are the indices along the two other axes in
 * increasing axis order. */
static inline int line_idx(int n, int d, int a, int b, int m) {
    if (d == 0) return sidx(n, m, a, b);
    if (d == 1) return sidx(n, a, m, b);
    return sidx(n, a, b, m);
}

/* Map x(xi) and dx/dxi of an element with (q+1)^3 equispaced geometry nodes
 * (x-fastest).  dxdr[c][d] = d x_c / d xi_d. */
static void geo_map(int q, const double *X /*[(q+1)^3][3]*/, const ld r[3],
                    ld x[3], ld dxdr[3][3]) {
    int m = q + 1;
    ld z[4];
    for (int a = 0; a < m; ++a) z[a] = -1.0L + 2.0L * a / q;
    ld N[3][4], dN[3][4];
    for (int d = 0; d < 3; ++d)
        for (int a = 0; a < m; ++a) {
            N[d][a] = lagr(m, z, a, r[d]);
            dN[d][a] = lagr_d(m, z, a, r[d]);
        }
    for (int c = 0; c < 3; ++c) {
        x[c] = 0;
        for (int d = 0; d < 3; ++d) dxdr[c][d] = 0;
    }
    for (int k = 0; k < m; ++k)
        for (int j = 0; j < m; ++j)
            for (int i = 0; i < m; ++i) {
                const double *P = X + 3 * (i + m * (j + m * k));
                ld w = N[0][i] * N[1][j] * N[2][k];
                ld w0 = dN[0][i] * N[1][j] * N[2][k];
                ld w1 = N[0][i] * dN[1][j] * N[2][k];
                ld w2 = N[0][i] * N[1][j] * dN[2][k];
                for (int c = 0; c < 3; ++c) {
                    x[c] += w * P[c];
                    dxdr[c][0] += w0 * P[c];
                    dxdr[c][1] += w1 * P[c];
                    dxdr[c][2] += w2 * P[c];
                }
            }
}

static void cross(const ld a[3], const ld b[3], ld c[3]) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

/* Contravariant (area-scaled) vectors a^d = |J| grad(xi_d): rows of |J| J^-1.
 * a^0 = x_eta x x_zeta, a^1 = x_zeta x x_xi, a^2 = x_xi x x_eta. */
static void contravariant(ld dxdr[3][3], ld S[3][3], ld *detJ) {
    ld t[3][3]; /* t[d] = column d of dx/dxi = x_{xi_d} */
    for (int d = 0; d < 3; ++d)
        for (int c = 0; c < 3; ++c) t[d][c] = dxdr[c][d];
    cross(t[1], t[2], S[0]);
    cross(t[2], t[0], S[1]);
    cross(t[0], t[1], S[2]);
    *detJ = t[0][0] * S[0][0] + t[0][1] * S[0][1] + t[0][2] * S[0][2];
}

/*
 * Element metrics at solution and flux points (Section "Numerical method":
 * the element-wise polynomial, its solution nodes x^s and flux nodes x^f with
 * outward normals n_i).  Metrics are evaluated pointwise from the mapping.
 *   xs  [ne][ns][3]          solution-point coordinates
 *   detJ[ne][ns]             Jacobian determinant
 *   S   [ne][ns][3][3]       S[d][c] = (|J| J^-1)_{d c}
 *   nf  [ne][6][n*n][3]      outward area-scaled normal at each flux point
 * Face f = 2*d + side (side 0 at xi_d = -1, side 1 at +1); face point
 * index a + n*b with (a,b) along the two other axes in increasing order.
 */
int orc_geometry_set(int ne, int q, const double *nodes, const int32_t *elem_nodes,
                     int p, int set, double *xs, double *detJ, double *S, double *nf) {
    if (q < 1 || q > 2 || p < 0 || (set == 1 && p < 1)) return ORC_EINVAL;
    int n = p + 1, ns = n * n * n, m = q + 1, ng = m * m * m;
    double xi[16];
    solution_points(set, n, xi, NULL);
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int e = 0; e < ne; ++e) {
        double X[27 * 3];
        for (int a = 0; a < ng; ++a)
            for (int c = 0; c < 3; ++c)
                X[3 * a + c] = nodes[3 * (int64_t)elem_nodes[(int64_t)e * ng + a] + c];
        for (int l = 0; l < n; ++l)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    int s = sidx(n, i, j, l);
                    ld r[3] = {xi[i], xi[j], xi[l]}, x[3], dx[3][3], Sm[3][3], dj;
                    geo_map(q, X, r, x, dx);
                    contravariant(dx, Sm, &dj);
                    if (!(dj > 0)) bad++;
                    for (int c = 0; c < 3; ++c) xs[((int64_t)e * ns + s) * 3 + c] = (double)x[c];
                    detJ[(int64_t)e * ns + s] = (double)dj;
                    for (int d = 0; d < 3; ++d)
                        for (int c = 0; c < 3; ++c)
                            S[(((int64_t)e * ns + s) * 3 + d) * 3 + c] = (double)Sm[d][c];
                }
        for (int d = 0; d < 3; ++d)
            for (int side = 0; side < 2; ++side)
                for (int b = 0; b < n; ++b)
                    for (int a = 0; a < n; ++a) {
                        ld r[3];
                        int ax0 = (d == 0) ? 1 : 0, ax1 = (d == 2) ? 1 : 2;
                        r[d] = side ? 1.0L : -1.0L;
                        r[ax0] = xi[a];
                        r[ax1] = xi[b];
                        ld x[3], dx[3][3], Sm[3][3], dj;
                        geo_map(q, X, r, x, dx);
                        contravariant(dx, Sm, &dj);
                        ld sg = side ? 1.0L : -1.0L;
                        for (int c = 0; c < 3; ++c)
                            nf[((((int64_t)e * 6 + 2 * d + side) * n * n) + a + n * b) * 3 + c] =
                                (double)(sg * Sm[d][c]);
                    }
    }
    return bad ? ORC_EINVAL : ORC_OK;
}

int orc_geometry(int ne, int q, const double *nodes, const int32_t *elem_nodes, int p, double *xs,
                 double *detJ, double *S, double *nf) {
    return orc_geometry_set(ne, q, nodes, elem_nodes, p, 0, xs, detJ, S, nf);
}

/* ------------------------------------------------------------------------ */
/* Problem description shared by the residual, collision and RK routines     */
/* ------------------------------------------------------------------------ */

typedef struct {
    int32_t ne, p, nu;
    const double *u;      /* [nu][3] velocity nodes */
    const double *w;      /* [nu] integration weights (operator M) */
    const double *detJ;   /* [ne][ns] */
    const double *S;      /* [ne][ns][3][3] */
    const double *nf;     /* [ne][6][n*n][3] */
    const int32_t *nbr_elem; /* [ne][6], -1 on a boundary */
    const int8_t *nbr_face;  /* [ne][6] */
    const int8_t *nbr_orient;/* [ne][6] */
    const int8_t *bc;        /* [ne][6]: 0 interior/periodic, 1 farfield, 2 diffuse wall,
                                3 specular (symmetry) wall */
    const double *f_inf;     /* [nu] farfield exterior state (bc 1) */
    double theta_w;          /* wall temperature (bc 2) */
    int32_t model;           /* 0 BGK, 1 ES-BGK, 2 collisionless (S = 0) */
    double Pr, mu_ref, theta_ref, omega;
    int32_t visc_law;        /* 0 power law, 1 Sutherland */
    double theta_s;
    double newton_tol;
    int32_t newton_max_iter;
    int32_t nv[3];           /* velocity nodes per axis, k = i + nv0 (j + nv1 l) */
    int32_t nodes;           /* solution points: 0 Gauss-Legendre, 1 Gauss-Lobatto */
    double delta;            /* internal degrees of freedom; > 0: the reduced pair (F, G) */
    int32_t ncomp;           /* 1 (monatomic f) or 2 (F then G per point, each nu values) */
    int32_t positivity;      /* 1: limit every RK stage value to f >= 0 (orc_positivity) */
} orc_problem;

/* Neighbour face point for own face point (a,b) under orientation code o:
 * bit0 swaps (a,b), bit1 reverses the first index, bit2 the second. */
static void orient_map(int n, int o, int a, int b, int *pa, int *pb) {
    int x = a, y = b;
    if (o & 1) { x = b; y = a; }
    if (o & 2) x = n - 1 - x;
    if (o & 4) y = n - 1 - y;
    *pa = x; *pb = y;
}

/*
 * Advective FR residual R = -div(u f) for every velocity node (Section
 * "Numerical method", eq. (transport) and the corrected flux with the upwind
 * common interface flux).  For each element and velocity u:
 *   F~_d(x_s) = (S(x_s) u)_d f(x_s)               transformed flux
 *   div_s     = sum_d sum_m D[i_d][m] F~_d(line)  (tensor-product derivative)
 *   at each flux point: f- = trace, u_n = u . n_scaled,
 *     F^I = u_n f- if u_n > 0 else u_n f+,  jump = F^I - u_n f-
 *     corr(line) += c_side[m] * jump
 *   R_s = -(div_s + corr_s) / |J|_s
 * Exterior states: neighbour trace; farfield f_inf; diffuse wall rho_w M_w;
 * specular wall: the interior trace at the mirrored velocity.
 */
int orc_residual(const orc_problem *P, const double *f, double *R) {
    int n = P->p + 1, ns = n * n * n, nfp = n * n, nu = P->nu, nut = nu * P->ncomp;
    double xi[16], D[256], lam[2][16], cv[2][16];
    if (orc_fr_ops_set(P->p, P->nodes, xi, D, lam[0], lam[1], cv[0], cv[1]) != ORC_OK) return ORC_EINVAL;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
    for (int e = 0; e < P->ne; ++e) {
        double *acc = (double *)calloc((size_t)ns * nut, sizeof(double));
        ld rwall[6 * 256];
        double *Ft = (double *)malloc((size_t)3 * ns * sizeof(double));
        double *fm = (double *)malloc((size_t)nu * sizeof(double));
        double *fp = (double *)malloc((size_t)nu * sizeof(double));
        double *un = (double *)malloc((size_t)nu * sizeof(double));
        if (!acc || !Ft || !fm || !fp || !un) { bad++; free(acc); free(Ft); free(fm); free(fp); free(un); continue; }
        const double *fe = f + (int64_t)e * ns * nut;
        /* every component (F, and G for the reduced pair) is advected alike;
         * kc runs over the state, k over the velocity nodes */
        for (int comp = 0; comp < P->ncomp; ++comp) {
        const int co = comp * nu;
        /* divergence of the transformed discontinuous flux */
        for (int k = 0; k < nu; ++k) {
            const double *uk = P->u + 3 * k;
            for (int s = 0; s < ns; ++s) {
                const double *Sm = P->S + ((int64_t)e * ns + s) * 9;
                for (int d = 0; d < 3; ++d)
                    Ft[d * ns + s] = (Sm[3 * d] * uk[0] + Sm[3 * d + 1] * uk[1] + Sm[3 * d + 2] * uk[2]) *
                                     fe[(int64_t)s * nut + co + k];
            }
            for (int l = 0; l < n; ++l)
                for (int j = 0; j < n; ++j)
                    for (int i = 0; i < n; ++i) {
                        ld dv = 0;
                        for (int m = 0; m < n; ++m) {
                            dv += (ld)D[i * n + m] * Ft[0 * ns + sidx(n, m, j, l)];
                            dv += (ld)D[j * n + m] * Ft[1 * ns + sidx(n, i, m, l)];
                            dv += (ld)D[l * n + m] * Ft[2 * ns + sidx(n, i, j, m)];
                        }
                        acc[(int64_t)sidx(n, i, j, l) * nut + co + k] = (double)dv;
                    }
        }
        /* interface corrections, face by face */
        for (int face = 0; face < 6; ++face) {
            int d = face / 2, side = face % 2;
            int nb = P->nbr_elem[e * 6 + face];
            for (int b = 0; b < n; ++b)
                for (int a = 0; a < n; ++a) {
                    const double *nv = P->nf + (((int64_t)e * 6 + face) * nfp + a + n * b) * 3;
                    for (int k = 0; k < nu; ++k) {
                        const double *uk = P->u + 3 * k;
                        ld t = 0;
                        for (int m = 0; m < n; ++m)
                            t += (ld)lam[side][m] * fe[(int64_t)line_idx(n, d, a, b, m) * nut + co + k];
                        fm[k] = (double)t;
                        un[k] = uk[0] * nv[0] + uk[1] * nv[1] + uk[2] * nv[2];
                    }
                    if (nb >= 0) {
                        int nface = P->nbr_face[e * 6 + face];
                        int nd = nface / 2, nside = nface % 2, pa, pb;
                        orient_map(n, P->nbr_orient[e * 6 + face], a, b, &pa, &pb);
                        const double *fn = f + (int64_t)nb * ns * nut;
                        for (int k = 0; k < nu; ++k) {
                            ld t = 0;
                            for (int m = 0; m < n; ++m)
                                t += (ld)lam[nside][m] * fn[(int64_t)line_idx(n, nd, pa, pb, m) * nut + co + k];
                            fp[k] = (double)t;
                        }
                    } else if (P->bc[e * 6 + face] == 1) {
                        for (int k = 0; k < nu; ++k) fp[k] = P->f_inf[co + k];
                    } else if (P->bc[e * 6 + face] == 2) {
                        /* diffuse isothermal wall, wall at rest: the exterior
                         * state is rho_w M(0, theta_w) with rho_w set so that
                         * the net mass flux through the wall vanishes */
                        ld out = 0, in = 0, tw = P->theta_w;
                        ld c0 = powl(2.0L * 3.14159265358979323846264338327950288L * tw, -1.5L);
                        ld rw;
                        if (comp == 0) {
                            for (int k = 0; k < nu; ++k) {
                                const double *uk = P->u + 3 * k;
                                if (un[k] > 0) out += (ld)P->w[k] * un[k] * fm[k];
                                else {
                                    ld uu = (ld)uk[0] * uk[0] + (ld)uk[1] * uk[1] + (ld)uk[2] * uk[2];
                                    in += (ld)P->w[k] * (-(ld)un[k]) * c0 * expl(-uu / (2 * tw));
                                }
                            }
                            rw = in > 0 ? out / in : 0;
                            rwall[face * nfp + a + n * b] = rw;
                        } else {
                            /* G: the mass flux of F sets the wall density; the
                             * wall emits delta theta_w / 2 times the F state */
                            rw = rwall[face * nfp + a + n * b] * 0.5L * P->delta * tw;
                        }
                        for (int k = 0; k < nu; ++k) {
                            const double *uk = P->u + 3 * k;
                            ld uu = (ld)uk[0] * uk[0] + (ld)uk[1] * uk[1] + (ld)uk[2] * uk[2];
                            fp[k] = (double)(rw * c0 * expl(-uu / (2 * tw)));
                        }
                    } else if (P->bc[e * 6 + face] == 3) {
                        /* specular wall: the exterior state at u is the
                         * interior trace at the mirror image of u in the wall
                         * plane; the plane must be normal to a coordinate
                         * axis and the grid symmetric in that axis, so the
                         * image is a node */
                        double nn = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
                        int ax = -1;
                        for (int c = 0; c < 3; ++c)
                            if (fabs(fabs(nv[c]) - nn) <= 1e-12 * nn) ax = c;
                        int str[3] = {1, P->nv[0], P->nv[0] * P->nv[1]};
                        int ok = ax >= 0;
                        if (ok) {
                            double lo = P->u[ax], hi = P->u[3 * (int64_t)(P->nv[ax] - 1) * str[ax] + ax];
                            ok = fabs(lo + hi) <= 1e-12 * (fabs(lo) > 1.0 ? fabs(lo) : 1.0);
                        }
                        if (!ok) {
                            bad++;
                            for (int k = 0; k < nu; ++k) fp[k] = fm[k];
                        } else {
                            for (int k = 0; k < nu; ++k) {
                                int idx = (k / str[ax]) % P->nv[ax];
                                int km = k + (P->nv[ax] - 1 - 2 * idx) * str[ax];
                                fp[k] = fm[km];
                            }
                        }
                    } else {
                        bad++;
                        for (int k = 0; k < nu; ++k) fp[k] = fm[k];
                    }
                    for (int k = 0; k < nu; ++k) {
                        double fup = un[k] > 0 ? fm[k] : fp[k];
                        double jump = un[k] * fup - un[k] * fm[k];
                        for (int m = 0; m < n; ++m)
                            acc[(int64_t)line_idx(n, d, a, b, m) * nut + co + k] += cv[side][m] * jump;
                    }
                }
        }
        } /* components */
        for (int s = 0; s < ns; ++s) {
            double dj = P->detJ[(int64_t)e * ns + s];
            for (int k = 0; k < nut; ++k)
                R[((int64_t)e * ns + s) * nut + k] = -acc[(int64_t)s * nut + k] / dj;
        }
        free(acc); free(Ft); free(fm); free(fp); free(un);
    }
    return bad ? ORC_EINVAL : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Velocity grid and moments                                                 */
/* ------------------------------------------------------------------------ */

/* Uniform Cartesian velocity grid with closed trapezoid weights (Section
 * "Numerical method": Cartesian velocity nodes on the velocity domain, M a
 * strictly positive trapezoid-rule integration operator).  Node
 * k = i + n0 (j + n1 l).  An axis with one node carries weight 1. */
int orc_vgrid(const int32_t n[3], const double umin[3], const double umax[3],
              double *u, double *w) {
    double *ax[3], *wx[3];
    for (int d = 0; d < 3; ++d) {
        if (n[d] < 1) return ORC_EINVAL;
        ax[d] = (double *)malloc(n[d] * sizeof(double));
        wx[d] = (double *)malloc(n[d] * sizeof(double));
        if (n[d] == 1) { ax[d][0] = umin[d]; wx[d][0] = 1.0; continue; }
        double du = (umax[d] - umin[d]) / (n[d] - 1);
        for (int i = 0; i < n[d]; ++i) {
            ax[d][i] = umin[d] + i * du;
            wx[d][i] = (i == 0 || i == n[d] - 1) ? 0.5 * du : du;
        }
    }
    for (int l = 0; l < n[2]; ++l)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                int64_t k = i + (int64_t)n[0] * (j + (int64_t)n[1] * l);
                u[3 * k] = ax[0][i]; u[3 * k + 1] = ax[1][j]; u[3 * k + 2] = ax[2][l];
                w[k] = wx[0][i] * wx[1][j] * wx[2][l];
            }
    for (int d = 0; d < 3; ++d) { free(ax[d]); free(wx[d]); }
    return ORC_OK;
}

/* Discrete moments Q = M.(f psi), psi = (1, u, |u|^2/2) (Section "Governing
 * equations", eq. (moments), monatomic; discretely by M). */
static void point_moments(int nu, const double *u, const double *w, const double *f, ld Q[5]) {
    for (int a = 0; a < 5; ++a) Q[a] = 0;
    for (int k = 0; k < nu; ++k) {
        ld wf = (ld)w[k] * f[k];
        ld ux = u[3 * k], uy = u[3 * k + 1], uz = u[3 * k + 2];
        Q[0] += wf;
        Q[1] += wf * ux;
        Q[2] += wf * uy;
        Q[3] += wf * uz;
        Q[4] += wf * 0.5L * (ux * ux + uy * uy + uz * uz);
    }
}

int orc_moments(int64_t npts, int nu, const double *u, const double *w, const double *f, double *Q) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < npts; ++i) {
        ld q[5];
        point_moments(nu, u, w, f + i * nu, q);
        for (int a = 0; a < 5; ++a) Q[5 * i + a] = (double)q[a];
    }
    return ORC_OK;
}

/* Pressure tensor Pi_ij = M.(f (u_i-U_i)(u_j-U_j)) (Section "Governing
 * equations", ES-BGK temperature tensor); order xx yy zz xy xz yz. */
static void point_pressure_tensor(int nu, const double *u, const double *w, const double *f,
                                  const ld U[3], ld Pi[6]) {
    for (int a = 0; a < 6; ++a) Pi[a] = 0;
    for (int k = 0; k < nu; ++k) {
        ld wf = (ld)w[k] * f[k];
        ld cx = u[3 * k] - U[0], cy = u[3 * k + 1] - U[1], cz = u[3 * k + 2] - U[2];
        Pi[0] += wf * cx * cx; Pi[1] += wf * cy * cy; Pi[2] += wf * cz * cz;
        Pi[3] += wf * cx * cy; Pi[4] += wf * cx * cz; Pi[5] += wf * cy * cz;
    }
}

int orc_pressure_tensor(int64_t npts, int nu, const double *u, const double *w,
                        const double *f, double *Pi) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < npts; ++i) {
        ld q[5], U[3], pi[6];
        point_moments(nu, u, w, f + i * nu, q);
        for (int d = 0; d < 3; ++d) U[d] = q[1 + d] / q[0];
        point_pressure_tensor(nu, u, w, f + i * nu, U, pi);
        for (int a = 0; a < 6; ++a) Pi[6 * i + a] = (double)pi[a];
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Conservative equilibrium (Section "Numerical method", eq.                 */
/* (discrete_compatibility)) and the BGK / ES-BGK collision                  */
/* ------------------------------------------------------------------------ */

/* Viscosity law: power law mu_ref (theta/theta_ref)^omega, or Sutherland's
 * law (Section "Governing equations"). */
double orc_viscosity(double theta, double mu_ref, double theta_ref, double omega,
                     int law, double theta_s) {
    if (law == 1)
        return mu_ref * pow(theta / theta_ref, 1.5) * (theta_ref + theta_s) / (theta + theta_s);
    return mu_ref * pow(theta / theta_ref, omega);
}

/* Solve the 5x5 system A x = b by Gaussian elimination with partial pivoting. */
static int solve5(ld A[5][5], ld b[5], ld x[5]) {
    ld M[5][6];
    for (int i = 0; i < 5; ++i) {
        for (int j = 0; j < 5; ++j) M[i][j] = A[i][j];
        M[i][5] = b[i];
    }
    for (int c = 0; c < 5; ++c) {
        int piv = c;
        for (int r = c + 1; r < 5; ++r)
            if (fabsl(M[r][c]) > fabsl(M[piv][c])) piv = r;
        if (M[piv][c] == 0) return -1;
        if (piv != c)
            for (int j = 0; j < 6; ++j) { ld t = M[c][j]; M[c][j] = M[piv][j]; M[piv][j] = t; }
        for (int r = c + 1; r < 5; ++r) {
            ld fct = M[r][c] / M[c][c];
            for (int j = c; j < 6; ++j) M[r][j] -= fct * M[c][j];
        }
    }
    for (int i = 4; i >= 0; --i) {
        ld s = M[i][5];
        for (int j = i + 1; j < 5; ++j) s -= M[i][j] * x[j];
        x[i] = s / M[i][i];
    }
    return 0;
}

/* Eigenvalues of a symmetric 3x3 matrix (closed form, trigonometric). */
static void sym3_eig(const ld A[3][3], ld ev[3]) {
    ld p1 = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    ld q = (A[0][0] + A[1][1] + A[2][2]) / 3;
    if (p1 == 0) { ev[0] = A[0][0]; ev[1] = A[1][1]; ev[2] = A[2][2]; return; }
    ld p2 = (A[0][0] - q) * (A[0][0] - q) + (A[1][1] - q) * (A[1][1] - q) +
            (A[2][2] - q) * (A[2][2] - q) + 2 * p1;
    ld p = sqrtl(p2 / 6);
    ld B[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) B[i][j] = (A[i][j] - (i == j ? q : 0)) / p;
    ld detB = B[0][0] * (B[1][1] * B[2][2] - B[1][2] * B[2][1]) -
              B[0][1] * (B[1][0] * B[2][2] - B[1][2] * B[2][0]) +
              B[0][2] * (B[1][0] * B[2][1] - B[1][1] * B[2][0]);
    ld r = detB / 2;
    ld phi = r <= -1 ? 3.14159265358979323846264338327950288L / 3 : (r >= 1 ? 0 : acosl(r) / 3);
    ev[0] = q + 2 * p * cosl(phi);
    ev[2] = q + 2 * p * cosl(phi + 2.0L * 3.14159265358979323846264338327950288L / 3);
    ev[1] = 3 * q - ev[0] - ev[2];
}

static ld det3(const ld A[3][3]) {
    return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
           A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
           A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

static void inv3(const ld A[3][3], ld B[3][3]) {
    ld d = det3(A);
    B[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / d;
    B[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / d;
    B[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / d;
    B[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / d;
    B[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / d;
    B[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / d;
    B[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / d;
    B[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / d;
    B[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / d;
}

/* Residual r(z) and Jacobian of the scaled compatibility system:
 *   sum_k wt_k psi(c_k) e_k(z) = (1, 0, 0, 0, 3/2),
 *   e_k = exp(z0 + z1 c1 + z2 c2 + z3 c3 - z4 q(c_k)/2),
 *   psi = (1, c, |c|^2/2), d e/d z = (1, c, -q/2) e. */
static void newton_system(int nu, const ld *c, const ld *wt, const ld *qf, const ld z[5],
                          ld r[5], ld J[5][5]) {
    for (int a = 0; a < 5; ++a) { r[a] = 0; for (int b = 0; b < 5; ++b) J[a][b] = 0; }
    for (int k = 0; k < nu; ++k) {
        const ld *ck = c + 3 * k;
        ld ex = expl(z[0] + z[1] * ck[0] + z[2] * ck[1] + z[3] * ck[2] - 0.5L * z[4] * qf[k]);
        ld we = wt[k] * ex;
        ld psi[5] = {1, ck[0], ck[1], ck[2], 0.5L * (ck[0] * ck[0] + ck[1] * ck[1] + ck[2] * ck[2])};
        ld phi[5] = {1, ck[0], ck[1], ck[2], -0.5L * qf[k]};
        for (int a = 0; a < 5; ++a) {
            r[a] += we * psi[a];
            for (int b = 0; b < 5; ++b) J[a][b] += we * psi[a] * phi[b];
        }
    }
    r[0] -= 1.0L;
    r[4] -= 1.5L;
}

static ld norm2(const ld r[5]) {
    ld s = 0;
    for (int a = 0; a < 5; ++a) s += r[a] * r[a];
    return sqrtl(s);
}
static ld normi(const ld r[5]) {
    ld s = 0;
    for (int a = 0; a < 5; ++a) s = fabsl(r[a]) > s ? fabsl(r[a]) : s;
    return s;
}

/*
 * Equilibrium at one solution point.  Given f over the velocity nodes:
 *   Q = M.(f psi); rho, U, theta = (2/3)(E/rho - |U|^2/2); P = rho theta;
 *   tau = mu(theta) / (Pr P)            (Pr taken as 1 for BGK);
 *   the modified equilibrium g' = g(Q') satisfies M.(g' psi) = Q exactly
 *   (discrete compatibility), with g' = rho theta^-3/2 exp(z0 + z.c - z4 q(c)/2),
 *   c = (u - U)/sqrt(theta); q(c) = |c|^2 (BGK) or c^T A c with
 *   A = theta T^-1, T = theta/Pr I + (1 - 1/Pr) Pi/rho (ES-BGK).
 * Outputs g[nu], tau, prim[5] = (rho', U', theta') of g' (theta' = theta/z4),
 * zout[5], iterations; returns a status code.
 */
/* Moments of the state at one point: (rho, rho U, E) with E the total energy
 * (for the reduced pair: the translational energy of F plus the integral of
 * G, Section "Governing equations"). */
static void state_moments(const orc_problem *P, const double *f, ld Q[5]) {
    point_moments(P->nu, P->u, P->w, f, Q);
    if (P->ncomp == 2)
        for (int k = 0; k < P->nu; ++k) Q[4] += (ld)P->w[k] * f[P->nu + k];
}

/* State moments [npts][5] of states with P's layout (F, or F then G). */
int orc_state_moments(const orc_problem *P, int64_t npts, const double *f, double *Q) {
    int64_t nut = (int64_t)P->nu * P->ncomp;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < npts; ++i) {
        ld q[5];
        state_moments(P, f + i * nut, q);
        for (int a = 0; a < 5; ++a) Q[5 * i + a] = (double)q[a];
    }
    return ORC_OK;
}

/* Temperature of a state with moments Q: E - rho |U|^2 / 2 = (3 + delta)/2 rho theta. */
static ld state_theta(const orc_problem *P, const ld Q[5]) {
    ld rho = Q[0], U[3] = {Q[1] / rho, Q[2] / rho, Q[3] / rho};
    ld dof = 3.0L + (P->ncomp == 2 ? (ld)P->delta : 0.0L);
    return (2.0L / dof) * (Q[4] / rho - 0.5L * (U[0] * U[0] + U[1] * U[1] + U[2] * U[2]));
}

static int point_equilibrium(const orc_problem *P, const double *f, double *g, double *tau,
                             double prim[5], double zout[5], int *iters, double *theta_eq) {
    int nu = P->nu;
    ld Q[5];
    state_moments(P, f, Q);
    *theta_eq = 0.0;
    ld rho = Q[0];
    *iters = 0;
    if (!(rho > 0) || !isfinite((double)rho)) {
        for (int k = 0; k < nu; ++k) g[k] = f[k];
        *tau = 1.0;
        for (int a = 0; a < 5; ++a) { prim[a] = 0; zout[a] = 0; }
        return ORC_NEWTON_NONREAL;
    }
    ld U[3] = {Q[1] / rho, Q[2] / rho, Q[3] / rho};
    ld theta = state_theta(P, Q);
    if (!(theta > 0) || !isfinite((double)theta)) {
        for (int k = 0; k < nu; ++k) g[k] = f[k];
        *tau = 1.0;
        for (int a = 0; a < 5; ++a) { prim[a] = 0; zout[a] = 0; }
        return ORC_NEWTON_NONREAL;
    }
    int status = ORC_NEWTON_OK;
    *theta_eq = (double)theta;
    double Pr = (P->model == 1) ? P->Pr : 1.0;
    double mu = orc_viscosity((double)theta, P->mu_ref, P->theta_ref, P->omega, P->visc_law, P->theta_s);
    *tau = mu / (Pr * (double)(rho * theta));

    ld A[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    if (P->model == 1) {
        ld pi[6];
        point_pressure_tensor(nu, P->u, P->w, f, U, pi);
        ld T[3][3], ev[3];
        ld a1 = theta / Pr, a2 = (1.0L - 1.0L / Pr) / rho;
        T[0][0] = a1 + a2 * pi[0]; T[1][1] = a1 + a2 * pi[1]; T[2][2] = a1 + a2 * pi[2];
        T[0][1] = T[1][0] = a2 * pi[3];
        T[0][2] = T[2][0] = a2 * pi[4];
        T[1][2] = T[2][1] = a2 * pi[5];
        sym3_eig(T, ev);
        ld lmin = ev[0] < ev[1] ? ev[0] : ev[1];
        lmin = lmin < ev[2] ? lmin : ev[2];
        if (lmin <= 1e-8L * theta) {
            status = ORC_NEWTON_ESGUARD;
        } else {
            ld Ti[3][3];
            inv3(T, Ti);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) A[i][j] = theta * Ti[i][j];
        }
    }
    /* scaled velocity nodes and weights: c = (u-U)/sqrt(theta), wt = w theta^-3/2; g = rho wt exp(...) */
    ld st = sqrtl(theta);
    ld *c = (ld *)malloc(sizeof(ld) * 3 * nu);
    ld *wt = (ld *)malloc(sizeof(ld) * nu);
    ld *qf = (ld *)malloc(sizeof(ld) * nu);
    for (int k = 0; k < nu; ++k) {
        for (int d = 0; d < 3; ++d) c[3 * k + d] = ((ld)P->u[3 * k + d] - U[d]) / st;
        wt[k] = (ld)P->w[k] / (theta * st);
        const ld *ck = c + 3 * k;
        ld qq = 0;
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) qq += ck[i] * A[i][j] * ck[j];
        qf[k] = qq;
    }
    /* cold guess: the continuous (ES-)Gaussian with the moments of f */
    const ld twopi = 2.0L * 3.14159265358979323846264338327950288L;
    ld zc[5] = {-1.5L * logl(twopi) + 0.5L * logl(det3(A)), 0, 0, 0, 1};
    ld z[5], r[5], J[5][5];
    for (int a = 0; a < 5; ++a) z[a] = zc[a];
    int conv = 0, it = 0, rej = 0; /* rej: rejected line-search trials over the whole solve */
    newton_system(nu, c, wt, qf, z, r, J);
    for (it = 0; it < P->newton_max_iter; ++it) {
        ld rn = norm2(r);
        ld rhs[5], dz[5];
        for (int a = 0; a < 5; ++a) rhs[a] = -r[a];
        if (solve5(J, rhs, dz)) break;
        if (normi(r) <= P->newton_tol) {
            /* converged: one extra full step makes the result independent
             * of the path taken to get here */
            for (int a = 0; a < 5; ++a) z[a] += dz[a];
            conv = 1;
            ++it;
            break;
        }
        /* backtracking: halve the step after each rejected trial; at most
         * 40 rejected trials in the whole solve */
        ld alpha = 1, zt[5], rt[5], Jt[5][5];
        int acc = 0;
        while (rej < 40) {
            for (int a = 0; a < 5; ++a) zt[a] = z[a] + alpha * dz[a];
            if (zt[4] > 0) {
                newton_system(nu, c, wt, qf, zt, rt, Jt);
                if (norm2(rt) < (1.0L - 1e-4L * alpha) * rn) { acc = 1; break; }
            }
            alpha *= 0.5L;
            ++rej;
        }
        if (!acc) break;
        for (int a = 0; a < 5; ++a) {
            z[a] = zt[a];
            r[a] = rt[a];
            for (int b = 0; b < 5; ++b) J[a][b] = Jt[a][b];
        }
    }
    *iters = it;
    if (!conv) {
        status = ORC_NEWTON_FALLBACK;
        for (int a = 0; a < 5; ++a) z[a] = zc[a];
    }
    ld pref = rho / (theta * st);
    for (int k = 0; k < nu; ++k) {
        const ld *ck = c + 3 * k;
        g[k] = (double)(pref * expl(z[0] + z[1] * ck[0] + z[2] * ck[1] + z[3] * ck[2] - 0.5L * z[4] * qf[k]));
    }
    /* primitive state of g': theta' = theta / z4, U' = U + sqrt(theta) A^-1 zlin / z4,
     * rho' = M.(g') with the continuous normalisation of the (ES-)Gaussian */
    ld Ai[3][3];
    inv3(A, Ai);
    ld m[3];
    for (int i = 0; i < 3; ++i)
        m[i] = (Ai[i][0] * z[1] + Ai[i][1] * z[2] + Ai[i][2] * z[3]) / z[4];
    ld mAm = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) mAm += m[i] * A[i][j] * m[j];
    ld detA = det3(A);
    prim[0] = (double)(rho * expl(z[0] + 0.5L * z[4] * mAm) * powl(twopi / z[4], 1.5L) / sqrtl(detA));
    for (int d = 0; d < 3; ++d) prim[1 + d] = (double)(U[d] + st * m[d]);
    prim[4] = (double)(theta / z[4]);
    for (int a = 0; a < 5; ++a) zout[a] = (double)z[a];
    free(c); free(wt); free(qf);
    return status;
}

/*
 * Collision source S = (g' - f) / tau at every solution point (Section
 * "Governing equations", BGK / ES-BGK operator; the modified equilibrium of
 * eq. (discrete_compatibility)).  Optional outputs (may be NULL):
 *   prim[npts][5] = (rho', U', theta'), zpar[npts][5], status[npts], iters[npts].
 * A non-realizable point (rho <= 0 or theta <= 0) gets S = 0.
 */
int orc_collide(const orc_problem *P, int64_t npts, const double *f, double *S,
                double *prim, double *zpar, int32_t *status, int32_t *iters) {
    int nu = P->nu, nut = nu * P->ncomp;
    if (P->model == 2) { /* collisionless: no source */
        memset(S, 0, sizeof(double) * (size_t)npts * nut);
        if (prim) memset(prim, 0, sizeof(double) * 5 * (size_t)npts);
        if (zpar) memset(zpar, 0, sizeof(double) * 5 * (size_t)npts);
        if (status) memset(status, 0, sizeof(int32_t) * (size_t)npts);
        if (iters) memset(iters, 0, sizeof(int32_t) * (size_t)npts);
        return ORC_OK;
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < npts; ++i) {
        double *g = (double *)malloc(sizeof(double) * nu);
        double tau, pr[5], zz[5], th;
        int it;
        const double *fi = f + i * nut;
        int st = point_equilibrium(P, fi, g, &tau, pr, zz, &it, &th);
        for (int k = 0; k < nu; ++k) S[i * nut + k] = (g[k] - fi[k]) / tau;
        /* G relaxes to delta theta / 2 times the equilibrium of F */
        for (int k = 0; k < nut - nu; ++k)
            S[i * nut + nu + k] = st == ORC_NEWTON_NONREAL ? 0.0 : (0.5 * P->delta * th * g[k] - fi[nu + k]) / tau;
        if (prim) for (int a = 0; a < 5; ++a) prim[5 * i + a] = pr[a];
        if (zpar) for (int a = 0; a < 5; ++a) zpar[5 * i + a] = zz[a];
        if (status) status[i] = st;
        if (iters) iters[i] = it;
        free(g);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Semi-discrete right-hand side, time stepping, diagnostics                 */
/* ------------------------------------------------------------------------ */

/* L(f) = R_advection(f) + S(f)  (Section "Numerical method": decoupled
 * advection per velocity node with the collision as nonlinear source). */
int orc_rhs(const orc_problem *P, const double *f, double *L) {
    int n = P->p + 1, ns = n * n * n;
    int64_t npts = (int64_t)P->ne * ns, tot = npts * P->nu * P->ncomp;
    double *S = (double *)malloc(sizeof(double) * tot);
    if (!S) return ORC_ENOMEM;
    int rc = orc_residual(P, f, L);
    if (P->model == 2) { free(S); return rc; } /* collisionless transport only */
    orc_collide(P, npts, f, S, NULL, NULL, NULL, NULL);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < tot; ++i) L[i] += S[i];
    free(S);
    return rc;
}

/*
 * One explicit step (the paper integrates explicitly in time; the scheme is
 * not named).  scheme 0: three-stage SSP Runge-Kutta in Shu-Osher form,
 *   f1 = f + dt L(f); f2 = 3/4 f + 1/4 (f1 + dt L(f1)); f = 1/3 f + 2/3 (f2 + dt L(f2)).
 * scheme 1: Williamson's three-stage low-storage (2N) scheme,
 *   A = (0, -5/9, -153/128), B = (1/3, 15/16, 8/15):
 *   dF = A_k dF + dt L(f); f = f + B_k dF.
 */
/*
 * Positivity limiter (Section "Numerical method": the scheme is the cited
 * positivity-preserving and conservative FR method; the limiter is the
 * scaling of Zhang and Shu).  For every element and every state value (each
 * velocity node of each component) separately:
 *   mean = sum_s W_s f_s / sum_s W_s,  W_s = (Gauss weight x |J|) at point s,
 *          the element integral of the value's polynomial over its volume;
 *   m    = the smallest value of the polynomial at the element's solution
 *          points and at its flux points (the face traces);
 *   if m < 0:  theta = mean / (mean - m) (0 if mean <= 0),
 *              f_s <- mean + theta (f_s - mean) at every solution point.
 * The mean, hence the element integral of every moment, is unchanged, and
 * the limited polynomial is nonnegative at all those points.
 */
int orc_positivity(const orc_problem *P, double *f) {
    const int n = P->p + 1, ns = n * n * n, nfp = n * n;
    const int nut = P->nu * P->ncomp;
    double xi[16], wq[16], xd[16], D[16 * 16], lam[2][16], cM[16], cP[16];
    solution_points(P->nodes, n, xi, wq);
    if (orc_fr_ops_set(P->p, P->nodes, xd, D, lam[0], lam[1], cM, cP)) return ORC_EINVAL;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < P->ne; ++e) {
        double Wt[729];  /* ns <= 9^3 */
        ld wsum = 0;
        for (int l = 0; l < n; ++l)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    const int s = sidx(n, i, j, l);
                    Wt[s] = wq[i] * wq[j] * wq[l] * P->detJ[e * ns + s];
                    wsum += Wt[s];
                }
        for (int k = 0; k < nut; ++k) {
            double *fe = f + (int64_t)e * ns * nut + k;  /* stride nut between points */
            ld acc = 0;
            double m = fe[0];
            for (int s = 0; s < ns; ++s) {
                acc += (ld)Wt[s] * fe[(int64_t)s * nut];
                if (fe[(int64_t)s * nut] < m) m = fe[(int64_t)s * nut];
            }
            for (int d = 0; d < 3; ++d)
                for (int side = 0; side < 2; ++side)
                    for (int q = 0; q < nfp; ++q) {
                        ld t = 0;
                        for (int mm = 0; mm < n; ++mm)
                            t += (ld)lam[side][mm] * fe[(int64_t)line_idx(n, d, q % n, q / n, mm) * nut];
                        if ((double)t < m) m = (double)t;
                    }
            if (!(m < 0.0)) continue;
            const double mean = (double)(acc / wsum);
            const double th = mean > 0.0 ? mean / (mean - m) : 0.0;
            for (int s = 0; s < ns; ++s) fe[(int64_t)s * nut] = mean + th * (fe[(int64_t)s * nut] - mean);
        }
    }
    return ORC_OK;
}

int orc_rk_step(const orc_problem *P, double *f, double dt, int scheme, int nsteps) {
    int n = P->p + 1, ns = n * n * n;
    int64_t tot = (int64_t)P->ne * ns * P->nu * P->ncomp;
    double *a = (double *)malloc(sizeof(double) * tot);
    double *b = (double *)malloc(sizeof(double) * tot);
    if (!a || !b) { free(a); free(b); return ORC_ENOMEM; }
    int rc = ORC_OK;
    for (int step = 0; step < nsteps; ++step) {
        if (scheme == 0) {
            rc |= orc_rhs(P, f, b);
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < tot; ++i) a[i] = f[i] + dt * b[i];
            if (P->positivity) rc |= orc_positivity(P, a);
            rc |= orc_rhs(P, a, b);
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < tot; ++i) a[i] = 0.75 * f[i] + 0.25 * (a[i] + dt * b[i]);
            if (P->positivity) rc |= orc_positivity(P, a);
            rc |= orc_rhs(P, a, b);
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < tot; ++i) f[i] = f[i] / 3.0 + 2.0 / 3.0 * (a[i] + dt * b[i]);
            if (P->positivity) rc |= orc_positivity(P, f);
        } else {
            const double A[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
            const double B[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
            for (int st = 0; st < 3; ++st) {
                rc |= orc_rhs(P, f, b);
#pragma omp parallel for schedule(static)
                for (int64_t i = 0; i < tot; ++i) {
                    a[i] = (st == 0 ? 0.0 : A[st] * a[i]) + dt * b[i];
                    f[i] += B[st] * a[i];
                }
                if (P->positivity) rc |= orc_positivity(P, f);
            }
        }
    }
    free(a); free(b);
    return rc;
}

/* Global conserved totals: integral over the domain of M.(f psi), with the
 * Gauss quadrature of the element (weights w_s |J|). */
int orc_totals(const orc_problem *P, const double *f, double *tot) {
    int n = P->p + 1, ns = n * n * n;
    double xi[16], wq[16];
    solution_points(P->nodes, n, xi, wq);
    int64_t npts = (int64_t)P->ne * ns;
    double *Q = (double *)malloc(sizeof(double) * 5 * npts);
    if (!Q) return ORC_ENOMEM;
    orc_state_moments(P, npts, f, Q);
    ld t[5] = {0, 0, 0, 0, 0};
    for (int64_t e = 0; e < P->ne; ++e)
        for (int l = 0; l < n; ++l)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    int64_t pt = e * ns + sidx(n, i, j, l);
                    ld wgt = (ld)wq[i] * wq[j] * wq[l] * P->detJ[pt];
                    for (int a = 0; a < 5; ++a) t[a] += wgt * Q[5 * pt + a];
                }
    for (int a = 0; a < 5; ++a) tot[a] = (double)t[a];
    free(Q);
    return ORC_OK;
}

/* Explicit time step: dt = CFL h_min / ((2p+1) max_k sum_d |u_k,d|), with the
 * element size measured as h = 2|J| / |a^d| over all solution points and
 * directions.  (The paper does not state a time-step rule.) */
double orc_dt(const orc_problem *P, double cfl) {
    int n = P->p + 1, ns = n * n * n;
    double hmin = 1e300, umax = 0;
    for (int64_t i = 0; i < (int64_t)P->ne * ns; ++i)
        for (int d = 0; d < 3; ++d) {
            const double *a = P->S + i * 9 + 3 * d;
            double h = 2.0 * P->detJ[i] / sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
            if (h < hmin) hmin = h;
        }
    for (int k = 0; k < P->nu; ++k) {
        double s = fabs(P->u[3 * k]) + fabs(P->u[3 * k + 1]) + fabs(P->u[3 * k + 2]);
        if (s > umax) umax = s;
    }
    return cfl * hmin / ((2 * P->p + 1) * umax);
}

/*
 * Density gradient-length local Knudsen number (Section "Results", the
 * continuum-breakdown indicator): Kn = lambda |grad rho| / rho with the local
 * mean free path lambda = (mu(theta) / rho) sqrt(pi / (2 theta)), from the
 * moments of f at every solution point.  grad rho is the gradient of the
 * element's solution polynomial of rho at the point (no interface term):
 * d rho / d x_c = (1/|J|) sum_d S[d][c] d rho / d xi_d, the xi derivatives
 * along lines with D.  A point with rho <= 0 or theta <= 0 gets Kn = 0.
 */
int orc_kn_gll(const orc_problem *P, const double *f, double *kn) {
    int n = P->p + 1, ns = n * n * n, nu = P->nu;
    double xi[16], D[256], lL[16], lR[16], cM[16], cP[16];
    if (orc_fr_ops_set(P->p, P->nodes, xi, D, lL, lR, cM, cP) != ORC_OK) return ORC_EINVAL;
#pragma omp parallel for schedule(static)
    for (int e = 0; e < P->ne; ++e) {
        ld Q[729][5];  /* ns <= 9^3 */
        for (int s = 0; s < ns; ++s)
            state_moments(P, f + ((int64_t)e * ns + s) * nu * P->ncomp, Q[s]);
        for (int l = 0; l < n; ++l)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) {
                    int s = sidx(n, i, j, l);
                    ld dr[3] = {0, 0, 0};
                    for (int m = 0; m < n; ++m) {
                        dr[0] += (ld)D[i * n + m] * Q[sidx(n, m, j, l)][0];
                        dr[1] += (ld)D[j * n + m] * Q[sidx(n, i, m, l)][0];
                        dr[2] += (ld)D[l * n + m] * Q[sidx(n, i, j, m)][0];
                    }
                    const double *Sm = P->S + ((int64_t)e * ns + s) * 9;
                    ld dj = P->detJ[(int64_t)e * ns + s], g2 = 0;
                    for (int c = 0; c < 3; ++c) {
                        ld gc = 0;
                        for (int d = 0; d < 3; ++d) gc += (ld)Sm[d * 3 + c] * dr[d];
                        gc /= dj;
                        g2 += gc * gc;
                    }
                    ld rho = Q[s][0];
                    ld th = state_theta(P, Q[s]);
                    double out = 0.0;
                    if (rho > 0 && th > 0) {
                        ld mu = orc_viscosity((double)th, P->mu_ref, P->theta_ref, P->omega, P->visc_law,
                                              P->theta_s);
                        ld lam = mu / rho * sqrtl(3.14159265358979323846264338327950288L / (2.0L * th));
                        out = (double)(lam * sqrtl(g2) / rho);
                    }
                    kn[(int64_t)e * ns + s] = out;
                }
    }
    return ORC_OK;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
