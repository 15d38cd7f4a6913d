// Host-side set-up of libfrdvm: FR operators, mesh checks, element metrics,
// velocity tables and device allocations.
//
// Section "Numerical method" of the paper: nodal degree-p polynomial per
// element on N_s solution nodes, flux nodes on the faces, correction
// functions that recover nodal DG, Cartesian velocity grid with a strictly
// positive trapezoid integration operator.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>

#include "frdvm_common.h"

using namespace frdvm;

namespace frdvm {

// Legendre P_n and its derivative at x (recurrence on n).
void legendre_eval(int n, double x, double &P, double &dP) {
    double pm = 1.0, pc = x;
    if (n == 0) { P = 1.0; dP = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        double pn = ((2.0 * k - 1.0) * x * pc - (k - 1.0) * pm) / k;
        pm = pc;
        pc = pn;
    }
    P = pc;
    dP = n * (x * pc - pm) / (x * x - 1.0);  // valid inside (-1,1)
}

// n-point Gauss-Legendre rule (ascending) by Newton on P_n.
void gauss_legendre_rule(int n, double *x, double *w) {
    for (int i = 0; i < n; ++i) {
        double t = std::cos(M_PI * (4.0 * (n - i) - 1.0) / (4.0 * n + 2.0));
        if (n == 1) t = 0.0;
        for (int it = 0; it < 60 && n > 1; ++it) {
            double P, dP;
            legendre_eval(n, t, P, dP);
            const double dx = P / dP;
            t -= dx;
            if (std::fabs(dx) < 1e-17) break;
        }
        double P, dP = 1.0;
        if (n > 1) legendre_eval(n, t, P, dP);
        x[i] = t;
        w[i] = 2.0 / ((1.0 - t * t) * dP * dP);
    }
}

// n-point Gauss-Lobatto rule (ascending): the end points and the extrema of
// P_{n-1}, weights 2 / (n (n-1) P_{n-1}^2).  The interior nodes are the
// roots of P'_{n-1}; Newton uses P'' from Legendre's equation.
void gauss_lobatto_rule(int n, double *x, double *w) {
    const int p = n - 1;
    for (int i = 0; i < n; ++i) {
        double t = -std::cos(M_PI * i / p);
        if (i > 0 && i < p) {
            for (int it = 0; it < 60; ++it) {
                double P, dP;
                legendre_eval(p, t, P, dP);
                const double d2P = (2.0 * t * dP - p * (p + 1.0) * P) / (1.0 - t * t);
                const double dx = dP / d2P;
                t -= dx;
                if (std::fabs(dx) < 1e-17) break;
            }
        }
        // P_p at the node by the three-term recurrence (the end points too)
        double pm = 1.0, pc = t;
        for (int k = 2; k <= p; ++k) {
            const double pn = ((2.0 * k - 1.0) * t * pc - (k - 1.0) * pm) / k;
            pm = pc;
            pc = pn;
        }
        x[i] = t;
        w[i] = 2.0 / (p * (p + 1.0) * pc * pc);
    }
}

}  // namespace frdvm

namespace {

// FR operators in barycentric form on Gauss-Legendre (nodes 0) or
// Gauss-Lobatto (nodes 1) points.  D: l_m'(xi_i) from barycentric weights;
// traces l_m(+-1); the correction derivative at xi_i for a unit jump on a
// face is the DG lifting M^-1 l(face) with the exact mass matrix
// M_ij = int l_i l_j (Huynh's g_DG correction reproduces nodal DG); on
// Gauss points M = diag(w), elsewhere it is assembled with an (n+1)-point
// Gauss rule and solved.
void build_ops(int p, int nodes, Ops1D &o) {
    const int n = p + 1;
    std::memset(&o, 0, sizeof(o));
    if (nodes == 1)
        gauss_lobatto_rule(n, o.xi, o.wq);
    else
        gauss_legendre_rule(n, o.xi, o.wq);
    double lamb[kMaxN];
    for (int j = 0; j < n; ++j) {
        double pr = 1.0;
        for (int m = 0; m < n; ++m)
            if (m != j) pr *= (o.xi[j] - o.xi[m]);
        lamb[j] = 1.0 / pr;
    }
    for (int i = 0; i < n; ++i) {
        double diag = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            const double v = (lamb[j] / lamb[i]) / (o.xi[i] - o.xi[j]);
            o.D[i * n + j] = v;
            diag -= v;
        }
        o.D[i * n + i] = diag;
    }
    // l_m(x) in barycentric form (exactly the unit vector at a node)
    auto basis = [&](double x, double *l) {
        for (int m = 0; m < n; ++m)
            if (x == o.xi[m]) {
                for (int r = 0; r < n; ++r) l[r] = r == m ? 1.0 : 0.0;
                return;
            }
        double den = 0.0;
        for (int m = 0; m < n; ++m) den += lamb[m] / (x - o.xi[m]);
        for (int m = 0; m < n; ++m) l[m] = (lamb[m] / (x - o.xi[m])) / den;
    };
    for (int side = 0; side < 2; ++side) basis(side ? 1.0 : -1.0, o.lam[side]);
    if (nodes != 1) {
        for (int side = 0; side < 2; ++side)
            for (int i = 0; i < n; ++i) o.corr[side][i] = o.lam[side][i] / o.wq[i];
        return;
    }
    double xg[kMaxN + 1], wg[kMaxN + 1], M[kMaxN][kMaxN + 2] = {};
    gauss_legendre_rule(n + 1, xg, wg);
    for (int g = 0; g < n + 1; ++g) {
        double l[kMaxN];
        basis(xg[g], l);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) M[i][j] += wg[g] * l[i] * l[j];
    }
    // solve M [c-, c+] = [l(-1), l(+1)] (symmetric positive definite, n <= 4)
    for (int i = 0; i < n; ++i) {
        M[i][n] = o.lam[0][i];
        M[i][n + 1] = o.lam[1][i];
    }
    for (int c = 0; c < n; ++c) {
        for (int r = c + 1; r < n; ++r) {
            const double fct = M[r][c] / M[c][c];
            for (int k = c; k < n + 2; ++k) M[r][k] -= fct * M[c][k];
        }
    }
    for (int side = 0; side < 2; ++side)
        for (int i = n - 1; i >= 0; --i) {
            double v = M[i][n + side];
            for (int k = i + 1; k < n; ++k) v -= M[i][k] * o.corr[side][k];
            o.corr[side][i] = v / M[i][i];
        }
}

template <typename T>
int dev_alloc(fr_dvm *h, T **p, size_t count) {
    if (*p) { hipFree(*p); *p = nullptr; }
    if (count == 0) return FR_DVM_OK;
    if (hipMalloc(reinterpret_cast<void **>(p), count * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        return h->fail(FR_DVM_ENOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
    }
    h->owned_bytes += count * sizeof(T);
    return FR_DVM_OK;
}

int upload(fr_dvm *h, void *dst, const void *src, size_t bytes) {
    if (hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess)
        return h->fail(FR_DVM_EHIP, "hipMemcpy upload failed");
    return FR_DVM_OK;
}

// Axis-aligned box check: the 8 corner nodes of element e span a box
// lo + (a0 hx, a1 hy, a2 hz).  Returns false otherwise.
bool element_box(const fr_dvm_mesh *m, int e, double lo[3], double hh[3]) {
    const int32_t *en = m->elem_nodes + (int64_t)e * 8;
    const double *x0 = m->nodes + 3 * (int64_t)en[0];
    const double *x7 = m->nodes + 3 * (int64_t)en[7];
    for (int d = 0; d < 3; ++d) { lo[d] = x0[d]; hh[d] = x7[d] - x0[d]; }
    double scale = std::max(std::fabs(hh[0]), std::max(std::fabs(hh[1]), std::fabs(hh[2])));
    for (int a = 0; a < 8; ++a) {
        const double *x = m->nodes + 3 * (int64_t)en[a];
        for (int d = 0; d < 3; ++d) {
            double want = lo[d] + ((a >> d) & 1) * hh[d];
            if (std::fabs(x[d] - want) > 1e-12 * (scale + std::fabs(lo[d]))) return false;
        }
    }
    return hh[0] > 0 && hh[1] > 0 && hh[2] > 0;
}

constexpr int kNotAxis = 1000;

// Straight axis-aligned boxes whose every face meets the opposite face of a
// neighbour under orientation 0 with the same face size (periodic boxes):
// constant metrics per element and the compact outflow-half traces.  Returns
// kNotAxis (nothing set) for any other mesh.
int setup_axis(fr_dvm *h, const fr_dvm_mesh *mesh, std::vector<double> &wq3J) {
    if (mesh->geom_order != 1) return kNotAxis;
    std::vector<double> hsz(3 * h->ne);
    for (int64_t e = 0; e < h->ne; ++e) {
        double lo[3], hh[3];
        if (!element_box(mesh, (int)e, lo, hh)) return kNotAxis;
        for (int d = 0; d < 3; ++d) hsz[3 * e + d] = hh[d];
    }
    for (int64_t e = 0; e < h->ne; ++e)
        for (int f = 0; f < 6; ++f) {
            const int32_t nb = mesh->nbr_elem[e * 6 + f];
            if (nb < 0 || mesh->nbr_face[e * 6 + f] != (f ^ 1) || mesh->nbr_orient[e * 6 + f] != 0) return kNotAxis;
            for (int t = 0; t < 3; ++t)
                if (t != f / 2 && std::fabs(hsz[3 * e + t] - hsz[3 * (int64_t)nb + t]) > 1e-12 * hsz[3 * e + t])
                    return kNotAxis;
        }
    h->axis_mode = true;
    h->h_gfac.resize(3 * h->ne);
    h->h_detJ.resize(h->ne * h->ns);
    double hmin = 1e300;
    for (int64_t e = 0; e < h->ne; ++e) {
        const double *hh = &hsz[3 * e];
        const double detJ = hh[0] * hh[1] * hh[2] / 8.0;
        for (int d = 0; d < 3; ++d) {
            h->h_gfac[3 * e + d] = 2.0 / hh[d];
            hmin = std::min(hmin, hh[d]);
        }
        int s = 0;
        for (int l = 0; l < h->n; ++l)
            for (int j = 0; j < h->n; ++j)
                for (int i = 0; i < h->n; ++i, ++s) {
                    h->h_detJ[e * h->ns + s] = detJ;
                    wq3J[e * h->ns + s] = h->ops.wq[i] * h->ops.wq[j] * h->ops.wq[l] * detJ;
                }
    }
    h->hmin = hmin;
    // trace layout: per face only the velocities that leave through it
    const VGrid &vg = h->vg;
    TraceLayout &tl = h->tl;
    int64_t off = 0;
    for (int f = 0; f < 6; ++f) {
        const int d = f / 2;
        const int64_t per = vg.nu / vg.nv[d];
        tl.cnt[f] = (f & 1) ? (int64_t)(vg.nv[d] - vg.pos_start[d]) * per : (int64_t)vg.neg_end[d] * per;
        tl.face_off[f] = off;
        off += tl.cnt[f] * h->nfp;
    }
    tl.elem = off * h->ncomp;  // one such layout per component of the state
    int rc;
    if (h->ncomp == 2 && (rc = dev_alloc(h, &h->d_gfp, (size_t)h->ne * h->ns))) return rc;
    if ((rc = dev_alloc(h, &h->d_gfac, 3 * h->ne))) return rc;
    return upload(h, h->d_gfac, h->h_gfac.data(), 3 * h->ne * sizeof(double));
}

// Lagrange basis of the equispaced nodes -1, 0, 1 (q = 2) or -1, 1 (q = 1)
// at x, and its derivative.
void shape_1d(int q, double x, double N[3], double dN[3]) {
    if (q == 1) {
        N[0] = 0.5 * (1.0 - x); N[1] = 0.5 * (1.0 + x);
        dN[0] = -0.5; dN[1] = 0.5;
    } else {
        N[0] = 0.5 * x * (x - 1.0); N[1] = 1.0 - x * x; N[2] = 0.5 * x * (x + 1.0);
        dN[0] = x - 0.5; dN[1] = -2.0 * x; dN[2] = x + 0.5;
    }
}

// Area-scaled contravariant vectors a^d = |J| grad xi_d (rows of the
// cofactor matrix of dx/dxi) and |J| at reference point r of an element
// with node coordinates X [(q+1)^3][3], x-fastest.
// Also the mapped position x(r) (pos, may be null).
void element_metrics(int q, const double *X, const double r[3], double a[3][3], double &detJ, double *pos = nullptr) {
    const int m = q + 1;
    double N[3][3], dN[3][3];
    for (int d = 0; d < 3; ++d) shape_1d(q, r[d], N[d], dN[d]);
    double t[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // t[d] = dx/dxi_d
    double x[3] = {0, 0, 0};
    for (int k = 0; k < m; ++k)
        for (int j = 0; j < m; ++j)
            for (int i = 0; i < m; ++i) {
                const double *P = X + 3 * (i + m * (j + m * k));
                const double g = N[0][i] * N[1][j] * N[2][k];
                const double g0 = dN[0][i] * N[1][j] * N[2][k];
                const double g1 = N[0][i] * dN[1][j] * N[2][k];
                const double g2 = N[0][i] * N[1][j] * dN[2][k];
                for (int c = 0; c < 3; ++c) {
                    x[c] += g * P[c];
                    t[0][c] += g0 * P[c];
                    t[1][c] += g1 * P[c];
                    t[2][c] += g2 * P[c];
                }
            }
    if (pos)
        for (int c = 0; c < 3; ++c) pos[c] = x[c];
    for (int d = 0; d < 3; ++d) {
        const double *u = t[(d + 1) % 3], *v = t[(d + 2) % 3];
        a[d][0] = u[1] * v[2] - u[2] * v[1];
        a[d][1] = u[2] * v[0] - u[0] * v[2];
        a[d][2] = u[0] * v[1] - u[1] * v[0];
    }
    detJ = t[0][0] * a[0][0] + t[0][1] * a[0][1] + t[0][2] * a[0][2];
}

// Own face point (a, b) -> the neighbour's face point under orientation
// code o (bit0 swaps the indices, bit1 reverses the first, bit2 the second).
void face_point_map(int n, int o, int a, int b, int &pa, int &pb) {
    pa = (o & 1) ? b : a;
    pb = (o & 1) ? a : b;
    if (o & 2) pa = n - 1 - pa;
    if (o & 4) pb = n - 1 - pb;
}

// Any hexahedral mesh (8- or 27-node, faces met under any orientation,
// farfield / wall boundaries): pointwise metrics at solution and flux points
// and full traces (every velocity at every flux point).
int setup_general(fr_dvm *h, const fr_dvm_mesh *mesh, std::vector<double> &wq3J) {
    const int q = mesh->geom_order, m = q + 1, ng = m * m * m, n = h->n, ns = h->ns, nfp = h->nfp;
    const int64_t ne = h->ne;
    h->axis_mode = false;
    std::vector<double> S((size_t)ne * ns * 9), ijac((size_t)ne * ns), nf((size_t)ne * 6 * nfp * 3);
    std::vector<double> xf((size_t)ne * 6 * nfp * 3);  // flux-point positions (face matching)
    h->h_detJ.resize(ne * ns);
    double hmin = 1e300;
    double X[27 * 3];
    for (int64_t e = 0; e < ne; ++e) {
        for (int g = 0; g < ng; ++g)
            for (int c = 0; c < 3; ++c) X[3 * g + c] = mesh->nodes[3 * (int64_t)mesh->elem_nodes[e * ng + g] + c];
        for (int l = 0, s = 0; l < n; ++l)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i, ++s) {
                    const double r[3] = {h->ops.xi[i], h->ops.xi[j], h->ops.xi[l]};
                    double a[3][3], J;
                    element_metrics(q, X, r, a, J);
                    if (!(J > 0)) return h->fail(FR_DVM_EINVAL, "non-positive Jacobian in element " + std::to_string(e));
                    const int64_t pt = e * ns + s;
                    for (int d = 0; d < 3; ++d) {
                        for (int c = 0; c < 3; ++c) S[pt * 9 + 3 * d + c] = a[d][c];
                        hmin = std::min(hmin, 2.0 * J / std::sqrt(a[d][0] * a[d][0] + a[d][1] * a[d][1] + a[d][2] * a[d][2]));
                    }
                    h->h_detJ[pt] = J;
                    ijac[pt] = 1.0 / J;
                    wq3J[pt] = h->ops.wq[i] * h->ops.wq[j] * h->ops.wq[l] * J;
                }
        for (int f = 0; f < 6; ++f) {
            const int d = f / 2, side = f & 1;
            const int t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
            for (int b = 0; b < n; ++b)
                for (int a = 0; a < n; ++a) {
                    double r[3];
                    r[d] = side ? 1.0 : -1.0;
                    r[t0] = h->ops.xi[a];
                    r[t1] = h->ops.xi[b];
                    double av[3][3], J;
                    element_metrics(q, X, r, av, J, &xf[((e * 6 + f) * nfp + a + n * b) * 3]);
                    for (int c = 0; c < 3; ++c)
                        nf[((e * 6 + f) * nfp + a + n * b) * 3 + c] = side ? av[d][c] : -av[d][c];
                }
        }
    }
    h->hmin = hmin;
    // conforming faces: at matched flux points the two outward normals
    // cancel and the two positions differ by one vector for the whole face
    // (zero, or the period of a periodic pair)
    std::vector<int32_t> conn((size_t)ne * 24), wall;
    for (int64_t e = 0; e < ne; ++e)
        for (int f = 0; f < 6; ++f) {
            const int32_t nb = mesh->nbr_elem[e * 6 + f];
            int32_t *c = &conn[(e * 6 + f) * 4];
            c[0] = nb;
            c[1] = nb >= 0 ? mesh->nbr_face[e * 6 + f] : 0;
            c[2] = nb >= 0 ? mesh->nbr_orient[e * 6 + f] : 0;
            c[3] = nb >= 0 ? 0 : mesh->bc[e * 6 + f];
            if (nb < 0) {
                if (c[3] == 2) wall.push_back((int32_t)(e * 6 + f));
                if (c[3] == 3) {
                    // specular: the face must be a plane normal to a coordinate
                    // axis (its mirror image of a node is then a node of a
                    // grid symmetric in that axis); the axis goes in c[2]
                    int ax = -1;
                    for (int t = 0; t < nfp; ++t) {
                        const double *u = &nf[((e * 6 + f) * nfp + t) * 3];
                        const double mag = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
                        int at = -1;
                        for (int cc = 0; cc < 3; ++cc)
                            if (std::fabs(std::fabs(u[cc]) - mag) <= 1e-12 * mag) at = cc;
                        if (at < 0 || (ax >= 0 && at != ax)) { ax = -2; break; }
                        ax = at;
                    }
                    const VGrid &vg = h->vg;
                    bool sym = ax >= 0;
                    if (sym) {
                        const double lo = vg.umin[ax], hi = vg.umin[ax] + (vg.nv[ax] - 1) * vg.du[ax];
                        sym = std::fabs(lo + hi) <= 1e-12 * std::max(1.0, std::fabs(lo));
                    }
                    if (!sym)
                        return h->fail(FR_DVM_EINVAL, "specular face " + std::to_string(f) + " of element " +
                                                          std::to_string(e) +
                                                          " is not a coordinate plane on a velocity grid symmetric in its axis");
                    c[2] = ax;
                }
                continue;
            }
            const double *x00 = &xf[((e * 6 + f) * nfp) * 3];
            double shift[3] = {0, 0, 0}, ext = 0;
            for (int t = 1; t < nfp; ++t)
                for (int c = 0; c < 3; ++c) ext = std::max(ext, std::fabs(x00[3 * t + c] - x00[c]));
            for (int b = 0; b < n; ++b)
                for (int a = 0; a < n; ++a) {
                    int pa, pb;
                    face_point_map(n, c[2], a, b, pa, pb);
                    const int64_t own = (e * 6 + f) * nfp + a + n * b;
                    const int64_t oth = ((int64_t)nb * 6 + c[1]) * nfp + pa + n * pb;
                    const double *u = &nf[own * 3], *v = &nf[oth * 3];
                    const double mag = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
                    const double gap = std::fabs(u[0] + v[0]) + std::fabs(u[1] + v[1]) + std::fabs(u[2] + v[2]);
                    double dev = 0;
                    for (int cc = 0; cc < 3; ++cc) {
                        const double dx = xf[oth * 3 + cc] - xf[own * 3 + cc];
                        if (a == 0 && b == 0) shift[cc] = dx;
                        dev = std::max(dev, std::fabs(dx - shift[cc]));
                    }
                    if (!(gap <= 1e-9 * mag) || !(dev <= 1e-9 * ext))
                        return h->fail(FR_DVM_EINVAL, "non-conforming face " + std::to_string(f) + " of element " + std::to_string(e));
                }
        }
    h->nwall = (int64_t)wall.size();
    h->tl.elem = (int64_t)6 * nfp * h->vg.nu * h->ncomp;
    int rc;
    if ((rc = dev_alloc(h, &h->d_S, S.size())) || (rc = upload(h, h->d_S, S.data(), S.size() * sizeof(double))))
        return rc;
    if ((rc = dev_alloc(h, &h->d_ijac, ijac.size())) || (rc = upload(h, h->d_ijac, ijac.data(), ijac.size() * sizeof(double))))
        return rc;
    if ((rc = dev_alloc(h, &h->d_nf, nf.size())) || (rc = upload(h, h->d_nf, nf.data(), nf.size() * sizeof(double))))
        return rc;
    {
        std::vector<float> Sf(S.begin(), S.end()), jf(ijac.begin(), ijac.end()), nff(nf.begin(), nf.end());
        if ((rc = dev_alloc(h, &h->d_Sf, Sf.size())) || (rc = upload(h, h->d_Sf, Sf.data(), Sf.size() * sizeof(float))) ||
            (rc = dev_alloc(h, &h->d_ijacf, jf.size())) || (rc = upload(h, h->d_ijacf, jf.data(), jf.size() * sizeof(float))) ||
            (rc = dev_alloc(h, &h->d_nff, nff.size())) || (rc = upload(h, h->d_nff, nff.data(), nff.size() * sizeof(float))))
            return rc;
    }
    if ((rc = dev_alloc(h, &h->d_conn, conn.size())) || (rc = upload(h, h->d_conn, conn.data(), conn.size() * sizeof(int32_t))))
        return rc;
    if (!wall.empty() && ((rc = dev_alloc(h, &h->d_wall, wall.size())) ||
                          (rc = upload(h, h->d_wall, wall.data(), wall.size() * sizeof(int32_t)))))
        return rc;
    if ((rc = dev_alloc(h, &h->d_rw, (size_t)ne * 6 * nfp))) return rc;
    if ((rc = dev_alloc(h, &h->d_mw, (size_t)h->vg.nu))) return rc;
    if (h->ncomp == 2 && (rc = dev_alloc(h, &h->d_gfp, (size_t)ne * ns))) return rc;
    return dev_alloc(h, &h->d_finf, (size_t)h->vg.nu * h->ncomp);
}

}  // namespace

extern "C" void fr_dvm_default_params(fr_dvm_params *p) {
    std::memset(p, 0, sizeof(*p));
    p->model = FR_DVM_BGK;
    p->prandtl = 1.0;
    p->mu_ref = 1e-3;
    p->theta_ref = 1.0;
    p->omega = 0.81;
    p->visc_law = 0;
    p->precision = FR_DVM_FP64;
    p->newton_tol = 1e-13;
    p->newton_max_iter = 50;
    p->guess = FR_DVM_GUESS_COLD;
    p->rk = FR_DVM_SSPRK3;
    p->farfield[0] = 1.0;
    p->farfield[4] = 1.0;
    p->theta_wall = 1.0;
    p->overlap = 0;
}

namespace frdvm {

// Velocity grid of a handle: nodes umin + i du per axis, trapezoid weights,
// the sign split of each axis.
int setup_vgrid(fr_dvm *h, const fr_dvm_vgrid *grid) {
    VGrid &vg = h->vg;
    int64_t nu = 1;
    for (int d = 0; d < 3; ++d) {
        int nd = grid->n[d];
        if (nd < 1 || nd > 64) return h->fail(FR_DVM_EINVAL, "velocity nodes per axis must be 1..64");
        if (nd > 1 && !(grid->umax[d] > grid->umin[d])) return h->fail(FR_DVM_EINVAL, "umax <= umin");
        vg.nv[d] = nd;
        vg.umin[d] = grid->umin[d];
        vg.du[d] = nd > 1 ? (grid->umax[d] - grid->umin[d]) / (nd - 1) : 0.0;
        h->wax[d].assign(nd, 1.0);
        for (int i = 0; i < nd && nd > 1; ++i) h->wax[d][i] = (i == 0 || i == nd - 1) ? 0.5 * vg.du[d] : vg.du[d];
        int ne_ = 0, ps = nd;
        for (int i = 0; i < nd; ++i) {
            double u = vg.umin[d] + i * vg.du[d];
            if (u < 0) ne_ = i + 1;
            if (u > 0 && ps == nd) ps = i;
        }
        vg.neg_end[d] = ne_;
        vg.pos_start[d] = ps;
        nu *= nd;
    }
    vg.nu = (int)nu;
    return FR_DVM_OK;
}

// Point weights (integral of each solution point's basis function, times
// |J|), the 1-D velocity weights and the statistics buffers on the device.
int finish_create(fr_dvm *h, const std::vector<double> &wq3J) {
    int rc;
    if ((rc = dev_alloc(h, &h->d_wq3J, h->ne * h->ns))) return rc;
    if ((rc = upload(h, h->d_wq3J, wq3J.data(), wq3J.size() * sizeof(double)))) return rc;
    std::vector<double> wax(3 * 64, 0.0);
    for (int d = 0; d < 3; ++d)
        for (int i = 0; i < h->vg.nv[d]; ++i) wax[64 * d + i] = h->wax[d][i];
    if ((rc = dev_alloc(h, &h->d_wax, 3 * 64))) return rc;
    if ((rc = upload(h, h->d_wax, wax.data(), wax.size() * sizeof(double)))) return rc;
    if ((rc = dev_alloc(h, &h->d_stats, kHist + 4))) return rc;
    if ((rc = dev_alloc(h, &h->d_maxres, 1))) return rc;
    if ((rc = dev_alloc(h, &h->d_tot, 8))) return rc;
    hipMemset(h->d_stats, 0, (kHist + 4) * sizeof(int64_t));
    hipMemset(h->d_maxres, 0, sizeof(double));
    return FR_DVM_OK;
}

}  // namespace frdvm

extern "C" int fr_dvm_create_gas(const fr_dvm_mesh *mesh, int order, int nodes, double delta,
                                 const fr_dvm_vgrid *grid, fr_dvm_t *out) {
    if (!out) return FR_DVM_EINVAL;
    *out = nullptr;
    if (!mesh || !grid || !mesh->nodes || !mesh->elem_nodes || !mesh->nbr_elem || !mesh->nbr_face ||
        !mesh->nbr_orient || !mesh->bc)
        return FR_DVM_EINVAL;
    fr_dvm *h = new fr_dvm();
    auto bail = [&](int rc) { *out = h; return rc; };  // keep the handle so the error is readable
    if (order < 1 || order > kMaxP) return bail(h->fail(FR_DVM_EUNSUPPORTED, "order must be 1..3"));
    if (mesh->n_elem <= 0 || mesh->n_nodes <= 0) return bail(h->fail(FR_DVM_EINVAL, "empty mesh"));
    hipGetDevice(&h->device);
    h->p = order;
    h->n = order + 1;
    h->ns = h->n * h->n * h->n;
    h->nfp = h->n * h->n;
    h->ne = mesh->n_elem;
    if (nodes != 0 && nodes != 1) return bail(h->fail(FR_DVM_EINVAL, "solution point set must be 0 or 1"));
    h->nodes = nodes;
    if (!(delta >= 0.0) || !std::isfinite(delta)) return bail(h->fail(FR_DVM_EINVAL, "delta must be finite and >= 0"));
    h->delta = delta;
    h->ncomp = delta > 0.0 ? 2 : 1;
    build_ops(order, nodes, h->ops);

    int rc = setup_vgrid(h, grid);
    if (rc) return bail(rc);

    // mesh: connectivity and tags
    if (mesh->geom_order != 1 && mesh->geom_order != 2) return bail(h->fail(FR_DVM_EINVAL, "geom_order must be 1 or 2"));
    const int ngeo = mesh->geom_order == 2 ? 27 : 8;
    for (int64_t i = 0; i < h->ne * ngeo; ++i)
        if (mesh->elem_nodes[i] < 0 || mesh->elem_nodes[i] >= mesh->n_nodes)
            return bail(h->fail(FR_DVM_EINVAL, "element node id out of range"));
    for (int64_t e = 0; e < h->ne; ++e)
        for (int f = 0; f < 6; ++f) {
            const int32_t nb = mesh->nbr_elem[e * 6 + f];
            if (nb < 0) {
                if (mesh->bc[e * 6 + f] < 1 || mesh->bc[e * 6 + f] > 3)
                    return bail(h->fail(FR_DVM_EINVAL, "face without neighbour and without a boundary tag"));
                continue;
            }
            if (nb >= h->ne) return bail(h->fail(FR_DVM_EINVAL, "neighbour id out of range"));
            const int nf = mesh->nbr_face[e * 6 + f], no = mesh->nbr_orient[e * 6 + f];
            if (nf < 0 || nf > 5 || no < 0 || no > 7) return bail(h->fail(FR_DVM_EINVAL, "neighbour face or orientation code out of range"));
            if (mesh->nbr_elem[(int64_t)nb * 6 + nf] != e || mesh->nbr_face[(int64_t)nb * 6 + nf] != f)
                return bail(h->fail(FR_DVM_EINVAL, "neighbour relation is not symmetric"));
        }
    std::vector<double> wq3J(h->ne * h->ns);
    rc = setup_axis(h, mesh, wq3J);
    if (rc == kNotAxis) rc = setup_general(h, mesh, wq3J);
    if (rc) return bail(rc);
    if (h->axis_mode) {
        // kept for a later move to the general-mesh path (positivity limiter)
        fr_dvm::MeshCopy &mc = h->mesh_copy;
        mc.n_elem = mesh->n_elem;
        mc.n_nodes = mesh->n_nodes;
        mc.geom_order = mesh->geom_order;
        mc.nodes.assign(mesh->nodes, mesh->nodes + 3 * (size_t)mesh->n_nodes);
        mc.elem_nodes.assign(mesh->elem_nodes, mesh->elem_nodes + (size_t)ngeo * mesh->n_elem);
        mc.nbr_elem.assign(mesh->nbr_elem, mesh->nbr_elem + 6 * (size_t)mesh->n_elem);
        mc.nbr_face.assign(mesh->nbr_face, mesh->nbr_face + 6 * (size_t)mesh->n_elem);
        mc.nbr_orient.assign(mesh->nbr_orient, mesh->nbr_orient + 6 * (size_t)mesh->n_elem);
        mc.bc.assign(mesh->bc, mesh->bc + 6 * (size_t)mesh->n_elem);
    }

    // device tables
    if ((rc = dev_alloc(h, &h->d_nbr, 6 * h->ne))) return bail(rc);
    if ((rc = upload(h, h->d_nbr, mesh->nbr_elem, 6 * h->ne * sizeof(int32_t)))) return bail(rc);
    if ((rc = finish_create(h, wq3J))) return bail(rc);
    *out = h;
    return FR_DVM_OK;
}

extern "C" int fr_dvm_create_nodes(const fr_dvm_mesh *mesh, int order, int nodes, const fr_dvm_vgrid *grid,
                                   fr_dvm_t *out) {
    return fr_dvm_create_gas(mesh, order, nodes, 0.0, grid, out);
}

extern "C" int fr_dvm_create(const fr_dvm_mesh *mesh, int order, const fr_dvm_vgrid *grid, fr_dvm_t *out) {
    return fr_dvm_create_gas(mesh, order, 0, 0.0, grid, out);
}

namespace {

// A box handle moves to the general-mesh path (the positivity limiter runs
// in the general stage kernel): pointwise metrics, full traces, its own
// boundary tables.  The box path's trace buffers are released here (their
// size depends on the path) and reallocated by the caller.
int move_to_general(fr_dvm *h) {
    const size_t es = h->prm.precision == FR_DVM_FP32 ? sizeof(float) : sizeof(double);  // trace values
    for (int b = 0; b < 2; ++b)
        if (h->d_tr[b]) {
            hipFree(h->d_tr[b]);
            h->d_tr[b] = nullptr;
            if (h->have_params) h->owned_bytes -= h->ne * h->tl.elem * es;
        }
    const fr_dvm::MeshCopy &mc = h->mesh_copy;
    fr_dvm_mesh m;
    m.n_elem = mc.n_elem;
    m.n_nodes = mc.n_nodes;
    m.geom_order = mc.geom_order;
    m.nodes = mc.nodes.data();
    m.elem_nodes = mc.elem_nodes.data();
    m.nbr_elem = mc.nbr_elem.data();
    m.nbr_face = mc.nbr_face.data();
    m.nbr_orient = mc.nbr_orient.data();
    m.bc = mc.bc.data();
    std::vector<double> wq3J(h->ne * h->ns);
    int rc = setup_general(h, &m, wq3J);
    if (!rc) rc = upload(h, h->d_wq3J, wq3J.data(), wq3J.size() * sizeof(double));
    return rc;
}

}  // namespace

extern "C" int fr_dvm_set_params(fr_dvm_t h, const fr_dvm_params *p) {
    if (!h || !p) return FR_DVM_EINVAL;
    if (p->model < 0 || p->model > 2) return h->fail(FR_DVM_EINVAL, "unknown model");
    if (p->precision != FR_DVM_FP64 && p->precision != FR_DVM_FP32 && p->precision != FR_DVM_FP32_DEV)
        return h->fail(FR_DVM_EINVAL, "unknown precision");
    if (p->precision == FR_DVM_FP32_DEV && (!h->axis_mode || p->positivity || h->ncomp != 1))
        return h->fail(FR_DVM_EUNSUPPORTED,
                       "FP32 deviation storage needs a periodic box mesh, a monatomic gas and no positivity limiter");
    if (p->model == FR_DVM_ESBGK && !(p->prandtl > 0)) return h->fail(FR_DVM_EINVAL, "Prandtl number must be positive");
    if (!(p->mu_ref > 0) && p->model != FR_DVM_FREE) return h->fail(FR_DVM_EINVAL, "mu_ref must be positive");
    if (p->newton_max_iter < 1 || p->newton_max_iter > 200) return h->fail(FR_DVM_EINVAL, "newton_max_iter out of range");
    if (p->rk != FR_DVM_SSPRK3 && p->rk != FR_DVM_LSRK3_2N) return h->fail(FR_DVM_EINVAL, "unknown RK scheme");
    if (p->guess < 0 || p->guess > 3) return h->fail(FR_DVM_EINVAL, "unknown guess mode");
    if (p->overlap != 0 && p->overlap != 1) return h->fail(FR_DVM_EINVAL, "overlap must be 0 or 1");
    if (p->positivity != 0 && p->positivity != 1) return h->fail(FR_DVM_EINVAL, "positivity must be 0 or 1");
    if (h->mx && p->positivity) return h->fail(FR_DVM_EUNSUPPORTED, "no positivity limiter on mixed meshes");
    bool realloc_all = !h->have_params || p->precision != h->prm.precision;
    if (p->positivity && h->axis_mode) {
        int rc0 = move_to_general(h);
        if (rc0) return rc0;
        realloc_all = true;
    }
    // moment record: rho, rho U, then E (BGK) or the raw second moments (ES),
    // plus the integral of G for the reduced pair
    int nmom = ((p->model == FR_DVM_ESBGK) ? 10 : 5) + (h->ncomp == 2 ? 1 : 0);
    bool realloc_mom = !h->have_params || nmom != h->nmom;
    // element size of the buffers allocated under the previous parameters
    const size_t es_old = h->have_params && h->prm.precision != FR_DVM_FP64 ? sizeof(float) : sizeof(double);
    // traces: in the precision of the stage arithmetic (FP32 for both FP32 forms)
    const size_t tes_old = h->have_params && h->prm.precision != FR_DVM_FP64 ? sizeof(float) : sizeof(double);
    h->prm = *p;
    h->nmom = nmom;
    h->stage_count = 0;
    size_t es = p->precision == FR_DVM_FP64 ? sizeof(double) : sizeof(float);
    size_t tes = p->precision != FR_DVM_FP64 ? sizeof(float) : sizeof(double);
    int64_t npts = h->ne * h->ns;
    int64_t nu = h->vg.nu * h->ncomp;  // state values per point
    // trace values per buffer
    const size_t trn = h->mx ? (size_t)h->mx->nfp * h->vg.nu : (size_t)(h->ne * h->tl.elem);
    int rc;
    if (realloc_all) {
        if (h->d_reg) { hipFree(h->d_reg); h->owned_bytes -= npts * nu * es_old; h->d_reg = nullptr; }
        for (int b = 0; b < 2; ++b)
            if (h->d_tr[b]) { hipFree(h->d_tr[b]); h->d_tr[b] = nullptr; h->owned_bytes -= trn * tes_old; }
        if (hipMalloc(&h->d_reg, npts * nu * es) != hipSuccess) { h->d_reg = nullptr; return h->fail(FR_DVM_ENOMEM, "register allocation failed"); }
        h->owned_bytes += npts * nu * es;
        for (int b = 0; b < 2; ++b) {
            if (hipMalloc(&h->d_tr[b], trn * tes) != hipSuccess) { h->d_tr[b] = nullptr; return h->fail(FR_DVM_ENOMEM, "trace allocation failed"); }
            h->owned_bytes += trn * tes;
        }
        if ((rc = dev_alloc(h, &h->d_eq, npts * kEqW))) return rc;
        for (int b = 0; b < 3; ++b)
            if ((rc = dev_alloc(h, &h->d_ref[b], p->precision == FR_DVM_FP32_DEV ? h->ne * kRefW : 0))) return rc;
        h->cur_ref = h->prev_ref = h->u0_ref = 0;
        if ((rc = dev_alloc(h, &h->d_z, npts * 5))) return rc;
        if ((rc = dev_alloc(h, &h->d_prim, npts * 5))) return rc;
        if ((rc = dev_alloc(h, &h->d_pt_iters, npts))) return rc;
        if ((rc = dev_alloc(h, &h->d_pt_evals, npts))) return rc;
        if ((rc = dev_alloc(h, &h->d_pt_status, npts))) return rc;
        if ((rc = dev_alloc(h, &h->d_pt_resid, npts))) return rc;
        h->zvalid = 0;
    }
    if (realloc_mom) {
        if ((rc = dev_alloc(h, &h->d_Q, npts * nmom))) return rc;
        // moment weights on the tensor velocity grid: along x per node
        // (w_x, w_x u_x, w_x u_x^2), per (y, z) row (W, W u_y, W u_z, W u_y^2,
        // W u_z^2, W u_y u_z) with W = w_y w_z
        const VGrid &vg = h->vg;
        std::vector<double> wx3((size_t)3 * vg.nv[0]), wrow((size_t)6 * vg.nv[1] * vg.nv[2]);
        for (int i = 0; i < vg.nv[0]; ++i) {
            const double ux = vg.umin[0] + i * vg.du[0], w = h->wax[0][i];
            wx3[3 * i] = w;
            wx3[3 * i + 1] = w * ux;
            wx3[3 * i + 2] = w * ux * ux;
        }
        for (int l = 0; l < vg.nv[2]; ++l)
            for (int j = 0; j < vg.nv[1]; ++j) {
                const double uy = vg.umin[1] + j * vg.du[1], uz = vg.umin[2] + l * vg.du[2];
                const double W = h->wax[1][j] * h->wax[2][l];
                double *o = &wrow[(size_t)6 * (j + (size_t)vg.nv[1] * l)];
                o[0] = W; o[1] = W * uy; o[2] = W * uz;
                o[3] = W * uy * uy; o[4] = W * uz * uz; o[5] = W * uy * uz;
            }
        if ((rc = dev_alloc(h, &h->d_wx3, wx3.size()))) return rc;
        if ((rc = upload(h, h->d_wx3, wx3.data(), wx3.size() * sizeof(double)))) return rc;
        if ((rc = dev_alloc(h, &h->d_wrow, wrow.size()))) return rc;
        if ((rc = upload(h, h->d_wrow, wrow.data(), wrow.size() * sizeof(double)))) return rc;
    }
    if (!h->axis_mode && !h->mx && (rc = gen_boundary_tables(h))) return rc;
    // verification switch: FRDVM_ES_DIRECT=1 makes the ES Newton use the
    // direct per-node sums instead of the factorised ones
    const char *ev = std::getenv("FRDVM_ES_DIRECT");
    h->es_direct = ev && ev[0] == '1';
    h->have_params = true;
    return FR_DVM_OK;
}

namespace frdvm {

// Wall Maxwellian of unit density at rest at theta_wall and the farfield
// Maxwellian (rho, U, theta) at every velocity node, in FP64 (boundary
// exteriors of the general-mesh path).
int gen_boundary_tables(fr_dvm *h) {
    const VGrid &vg = h->vg;
    std::vector<double> mw(vg.nu), fi((size_t)vg.nu * h->ncomp);
    const double kPi = 3.14159265358979323846;
    const double tw = h->prm.theta_wall, *F = h->prm.farfield;
    for (int64_t k = 0; k < vg.nu; ++k) {
        const int i = (int)(k % vg.nv[0]), j = (int)((k / vg.nv[0]) % vg.nv[1]);
        const int l = (int)(k / ((int64_t)vg.nv[0] * vg.nv[1]));
        const double u[3] = {vg.umin[0] + i * vg.du[0], vg.umin[1] + j * vg.du[1], vg.umin[2] + l * vg.du[2]};
        const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        mw[k] = tw > 0 ? std::pow(2.0 * kPi * tw, -1.5) * std::exp(-uu / (2.0 * tw)) : 0.0;
        const double c0 = u[0] - F[1], c1 = u[1] - F[2], c2 = u[2] - F[3];
        fi[k] = (F[0] > 0 && F[4] > 0)
                    ? F[0] * std::pow(2.0 * kPi * F[4], -1.5) * std::exp(-(c0 * c0 + c1 * c1 + c2 * c2) / (2.0 * F[4]))
                    : 0.0;
    }
    // the pair's farfield G: delta theta_inf / 2 times the farfield F
    for (int64_t k = 0; k < (int64_t)vg.nu * (h->ncomp - 1); ++k) fi[vg.nu + k] = 0.5 * h->delta * F[4] * fi[k];
    int rc = upload(h, h->d_mw, mw.data(), mw.size() * sizeof(double));
    if (!rc) rc = upload(h, h->d_finf, fi.data(), fi.size() * sizeof(double));
    return rc;
}

}  // namespace frdvm

extern "C" int fr_dvm_set_stream(fr_dvm_t h, void *stream) {
    if (!h) return FR_DVM_EINVAL;
    h->stream = reinterpret_cast<hipStream_t>(stream);
    return FR_DVM_OK;
}

extern "C" int fr_dvm_sizes(fr_dvm_t h, int64_t *n_elem, int32_t *ns, int32_t *nf, int32_t *nu, size_t *ws) {
    if (!h) return FR_DVM_EINVAL;
    if (n_elem) *n_elem = h->ne;
    if (ns) *ns = h->ns;
    if (nf) *nf = 6 * h->nfp;
    if (nu) *nu = h->vg.nu;
    if (ws) *ws = h->owned_bytes;
    return FR_DVM_OK;
}

extern "C" int fr_dvm_velocity_nodes(fr_dvm_t h, double *u, double *w) {
    if (!h) return FR_DVM_EINVAL;
    const VGrid &vg = h->vg;
    for (int64_t k = 0; k < vg.nu; ++k) {
        int i = (int)(k % vg.nv[0]), j = (int)((k / vg.nv[0]) % vg.nv[1]), l = (int)(k / ((int64_t)vg.nv[0] * vg.nv[1]));
        if (u) {
            u[3 * k] = vg.umin[0] + i * vg.du[0];
            u[3 * k + 1] = vg.umin[1] + j * vg.du[1];
            u[3 * k + 2] = vg.umin[2] + l * vg.du[2];
        }
        if (w) w[k] = h->wax[0][i] * h->wax[1][j] * h->wax[2][l];
    }
    return FR_DVM_OK;
}

extern "C" int fr_dvm_dt(fr_dvm_t h, double cfl, double *dt) {
    if (!h || !dt || !(cfl > 0)) return FR_DVM_EINVAL;
    double um = 0;
    for (int d = 0; d < 3; ++d) {
        double a = std::fabs(h->vg.umin[d]), b = std::fabs(h->vg.umin[d] + (h->vg.nv[d] - 1) * h->vg.du[d]);
        um += std::max(a, b);
    }
    *dt = cfl * h->hmin / ((2 * h->p + 1) * um);
    return FR_DVM_OK;
}

extern "C" const char *fr_dvm_last_error(fr_dvm_t h) { return h ? h->err.c_str() : "null handle"; }

extern "C" void fr_dvm_destroy(fr_dvm_t h) {
    if (!h) return;
    if (h->stream) hipStreamSynchronize(h->stream); else hipDeviceSynchronize();
    free_mixed(h);
    void *ptrs[] = {h->d_gfac, h->d_nbr, h->d_wq3J, h->d_wx3, h->d_wrow, h->d_wax, h->d_reg, h->d_tr[0], h->d_tr[1],
                    h->d_Q, h->d_eq, h->d_ref[0], h->d_ref[1], h->d_ref[2], h->d_z, h->d_prim, h->d_stats, h->d_maxres, h->d_tot, h->d_mlp,
                    h->d_mlp_x, h->d_mlp_work, h->d_mlp_dz, h->d_pt_iters, h->d_pt_evals, h->d_pt_status,
                    h->d_pt_resid, h->d_S, h->d_ijac, h->d_nf, h->d_conn, h->d_wall, h->d_rw, h->d_mw,
                    h->d_finf, h->d_Sf, h->d_ijacf, h->d_nff, h->d_gfp};
    for (void *p : ptrs)
        if (p) hipFree(p);
    for (auto &r : h->prof_recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    if (h->aux) {
        (void)hipStreamSynchronize(h->aux);
        (void)hipStreamDestroy(h->aux);
    }
    for (int i = 0; i < 2; ++i) {
        if (h->ev_stage[i]) (void)hipEventDestroy(h->ev_stage[i]);
        if (h->ev_newton[i]) (void)hipEventDestroy(h->ev_newton[i]);
    }
    delete h;
}
