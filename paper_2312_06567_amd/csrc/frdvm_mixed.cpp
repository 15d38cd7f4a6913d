// Set-up of mixed meshes of straight hexahedra, prisms and tetrahedra
// (fr_dvm_create_mixed, Section "Implementation & problem setup": the paper's
// prisms and tetrahedra, alpha-optimised points on simplices, Gauss-Lobatto
// points on tensor-product elements).
//
// Per element type the nodal operators of FR with the DG-recovering
// correction (Section "Numerical method"): with l_i the Lagrange functions of
// the solution points, D_a[i][j] = d l_j / d xi_a (x_i), and the correction of
// a unit jump at face point t of face f, lift[i][t] = (M^-1 E_f)[i][t] with
// M_ij = int l_i l_j over the element and E_f[i][t] = int over f of
// l_i l_(node of t), stored by face point (row t: the column of face point
// t, contiguous, so that a kernel reading it for one face point reads
// consecutive entries).  Derivation: a basis of Legendre products
// P_a(xi) P_b(eta) P_c(zeta) over the type's exponent set (total degree <= p
// on the tetrahedron; <= p in (xi, eta) times <= p in zeta on the prism;
// <= p per axis on the hexahedron), its Vandermonde matrix at the solution
// points inverted, and the integrals by Gauss-Legendre rules collapsed onto
// the triangle and the tetrahedron (exact for the degree 2p integrands).
//
// Geometry: every element is the affine image x = x0 + A (xi + 1) of its
// reference element; per element dxi/dx = A^-1, the unit outward normal of
// each face and |J_face| / |J| (physical over reference face area, over the
// volume ratio).  The face points of neighbouring faces are matched by
// position (modulo the domain's period).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "frdvm_common.h"

using namespace frdvm;

namespace {

using V3 = std::array<double, 3>;

const double kRefV[3][8][3] = {
    {{-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {1, 1, -1}, {-1, -1, 1}, {1, -1, 1}, {-1, 1, 1}, {1, 1, 1}},
    {{-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {-1, -1, 1}, {1, -1, 1}, {-1, 1, 1}},
    {{-1, -1, -1}, {1, -1, -1}, {-1, 1, -1}, {-1, -1, 1}},
};
const int kNV[3] = {8, 6, 4};
const int kNF[3] = {6, 5, 4};
// face vertices (-1: a triangle)
const int kFaceV[3][6][4] = {
    {{0, 2, 4, 6}, {1, 3, 5, 7}, {0, 1, 4, 5}, {2, 3, 6, 7}, {0, 1, 2, 3}, {4, 5, 6, 7}},
    {{0, 1, 2, -1}, {3, 4, 5, -1}, {0, 1, 4, 3}, {1, 2, 5, 4}, {2, 0, 3, 5}},
    {{0, 1, 2, -1}, {0, 1, 3, -1}, {1, 2, 3, -1}, {0, 2, 3, -1}},
};
// vertices spanning the affine map from vertex 0
const int kAxes[3][3] = {{1, 2, 4}, {1, 2, 3}, {1, 2, 3}};

V3 sub(const V3 &a, const V3 &b) { return {a[0] - b[0], a[1] - b[1], a[2] - b[2]}; }
V3 cross(const V3 &a, const V3 &b) {
    return {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
}
double dot(const V3 &a, const V3 &b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
double norm(const V3 &a) { return std::sqrt(dot(a, a)); }

std::vector<double> lobatto_points(int p) {
    std::vector<double> x(p + 1), w(p + 1);
    gauss_lobatto_rule(p + 1, x.data(), w.data());
    return x;
}

// Solution points of the reference triangle (dim 2) / tetrahedron (dim 3),
// p <= 3: barycentric (i, j[, k]) / p, points on an edge moved to the
// Gauss-Lobatto position along it (the warp & blend points for p <= 3).
std::vector<V3> simplex_points(int p, int dim) {
    const std::vector<double> gl = lobatto_points(p);
    std::vector<V3> out;
    auto emit = [&](int i, int j, int k) {
        double lam[4] = {double(p - i - j - k) / p, double(i) / p, double(j) / p, double(k) / p};
        int nz[4], c = 0;
        for (int a = 0; a <= dim; ++a)
            if (lam[a] > 0) nz[c++] = a;
        if (c == 2) {
            const int m = (int)std::lround(lam[nz[1]] * p);
            lam[nz[1]] = 0.5 * (1.0 + gl[m]);
            lam[nz[0]] = 1.0 - lam[nz[1]];
        }
        V3 x{0, 0, 0};
        for (int a = 0; a <= dim; ++a)
            for (int d = 0; d < 3; ++d) x[d] += lam[a] * kRefV[2][a][d];
        if (dim == 2) x[2] = 0.0;
        out.push_back(x);
    };
    if (dim == 2) {
        for (int j = 0; j <= p; ++j)
            for (int i = 0; i + j <= p; ++i) emit(i, j, 0);
    } else {
        for (int k = 0; k <= p; ++k)
            for (int j = 0; j + k <= p; ++j)
                for (int i = 0; i + j + k <= p; ++i) emit(i, j, k);
    }
    return out;
}

std::vector<V3> ref_points(int t, int p) {
    const std::vector<double> gl = lobatto_points(p);
    std::vector<V3> out;
    if (t == FR_DVM_HEX) {
        for (double z : gl)
            for (double y : gl)
                for (double x : gl) out.push_back({x, y, z});
    } else if (t == FR_DVM_PRISM) {
        const std::vector<V3> tri = simplex_points(p, 2);
        for (double z : gl)
            for (const V3 &q : tri) out.push_back({q[0], q[1], z});
    } else {
        out = simplex_points(p, 3);
    }
    return out;
}

std::vector<std::array<int, 3>> exponents(int t, int p) {
    std::vector<std::array<int, 3>> ex;
    for (int c = 0; c <= p; ++c)
        for (int b = 0; b <= p; ++b)
            for (int a = 0; a <= p; ++a) {
                if (t == FR_DVM_PRISM && a + b > p) continue;
                if (t == FR_DVM_TET && a + b + c > p) continue;
                ex.push_back({a, b, c});
            }
    return ex;
}

// Legendre P_0..P_p and their derivatives at x.
void legendre_all(int p, double x, double *P, double *dP) {
    P[0] = 1.0;
    dP[0] = 0.0;
    if (p >= 1) {
        P[1] = x;
        dP[1] = 1.0;
    }
    for (int n = 2; n <= p; ++n) {
        P[n] = ((2.0 * n - 1.0) * x * P[n - 1] - (n - 1.0) * P[n - 2]) / n;
        dP[n] = dP[n - 2] + (2.0 * n - 1.0) * P[n - 1];
    }
}

// Basis values (and gradients) of the Legendre-product basis at x.
void basis(const std::vector<std::array<int, 3>> &ex, int p, const V3 &x, double *phi, double (*grad)[3]) {
    double P[3][kMaxN], dP[3][kMaxN];
    for (int d = 0; d < 3; ++d) legendre_all(p, x[d], P[d], dP[d]);
    for (size_t m = 0; m < ex.size(); ++m) {
        const int a = ex[m][0], b = ex[m][1], c = ex[m][2];
        phi[m] = P[0][a] * P[1][b] * P[2][c];
        if (grad) {
            grad[m][0] = dP[0][a] * P[1][b] * P[2][c];
            grad[m][1] = P[0][a] * dP[1][b] * P[2][c];
            grad[m][2] = P[0][a] * P[1][b] * dP[2][c];
        }
    }
}

// In-place inverse of a dense n x n matrix (Gauss-Jordan, partial pivoting).
bool invert(std::vector<double> &A, int n) {
    std::vector<double> I(n * n, 0.0);
    for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
        if (std::fabs(A[piv * n + c]) < 1e-300) return false;
        if (piv != c)
            for (int k = 0; k < n; ++k) {
                std::swap(A[piv * n + k], A[c * n + k]);
                std::swap(I[piv * n + k], I[c * n + k]);
            }
        const double inv = 1.0 / A[c * n + c];
        for (int k = 0; k < n; ++k) {
            A[c * n + k] *= inv;
            I[c * n + k] *= inv;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double f = A[r * n + c];
            if (f == 0.0) continue;
            for (int k = 0; k < n; ++k) {
                A[r * n + k] -= f * A[c * n + k];
                I[r * n + k] -= f * I[c * n + k];
            }
        }
    }
    A.swap(I);
    return true;
}

// Volume rule of the reference element: Gauss-Legendre in each direction,
// collapsed (Duffy) onto the triangle of the prism and onto the tetrahedron.
void volume_rule(int t, int n, std::vector<V3> &x, std::vector<double> &w) {
    std::vector<double> g(n), gw(n);
    gauss_legendre_rule(n, g.data(), gw.data());
    for (int k = 0; k < n; ++k)
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                const double a = g[i], b = g[j], c = g[k];
                double wt = gw[i] * gw[j] * gw[k];
                if (t == FR_DVM_HEX) {
                    x.push_back({a, b, c});
                } else if (t == FR_DVM_PRISM) {
                    // triangle: eta = b, xi = (1 + a)(1 - eta)/2 - 1
                    x.push_back({0.5 * (1.0 + a) * (1.0 - b) - 1.0, b, c});
                    wt *= 0.5 * (1.0 - b);
                } else {
                    const double zt = c, et = 0.5 * (1.0 + b) * (1.0 - zt) - 1.0;
                    x.push_back({0.5 * (1.0 + a) * (-et - zt) - 1.0, et, zt});
                    wt *= 0.5 * (1.0 - zt) * 0.5 * (-et - zt);
                }
                w.push_back(wt);
            }
}

// Corner and the two edge vectors of a parallelogram given by 4 vertices in
// any order (the vertex farthest from the first is the opposite corner).
void quad_edges(const V3 v[4], V3 &e1, V3 &e2) {
    int far = 1;
    for (int i = 2; i < 4; ++i)
        if (norm(sub(v[i], v[0])) > norm(sub(v[far], v[0]))) far = i;
    int a = -1, b = -1;
    for (int i = 1; i < 4; ++i)
        if (i != far) (a < 0 ? a : b) = i;
    e1 = sub(v[a], v[0]);
    e2 = sub(v[b], v[0]);
}

double face_area(const V3 *v, bool quad) {
    if (!quad) return 0.5 * norm(cross(sub(v[1], v[0]), sub(v[2], v[0])));
    V3 e1, e2;
    quad_edges(v, e1, e2);
    return norm(cross(e1, e2));
}

// Rule on a planar face (reference surface measure): collapsed
// Gauss-Legendre on a triangle, tensor Gauss-Legendre on a parallelogram.
void face_rule(const V3 *v, bool quad, int n, std::vector<V3> &x, std::vector<double> &w) {
    std::vector<double> g(n), gw(n);
    gauss_legendre_rule(n, g.data(), gw.data());
    V3 e1, e2;
    double meas;
    if (quad) {
        quad_edges(v, e1, e2);
        meas = norm(cross(e1, e2));
    } else {
        e1 = sub(v[1], v[0]);
        e2 = sub(v[2], v[0]);
        meas = norm(cross(e1, e2));
    }
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            double u = 0.5 * (1.0 + g[i]), s = 0.5 * (1.0 + g[j]), wt = 0.25 * gw[i] * gw[j] * meas;
            if (!quad) {
                s *= 1.0 - u;
                wt *= 1.0 - u;
            }
            x.push_back({v[0][0] + u * e1[0] + s * e2[0], v[0][1] + u * e1[1] + s * e2[1], v[0][2] + u * e1[2] + s * e2[2]});
            w.push_back(wt);
        }
}

std::vector<V3> ref_verts(int t) {
    std::vector<V3> v(kNV[t]);
    for (int i = 0; i < kNV[t]; ++i) v[i] = {kRefV[t][i][0], kRefV[t][i][1], kRefV[t][i][2]};
    return v;
}

// The prism's points are the triangle's points on every Gauss-Lobatto layer
// (point m + nt k, nt triangle points, k the layer) and its space is
// P_p(triangle) x P_p(line), so its nodal basis is the product of the two
// Lagrange bases and its operators inherit the product structure: the
// in-plane derivatives couple only points of one layer, the axial one only
// points of one column; a bottom or top face point (that column's end)
// lifts onto its column, a side face point (edge point e on layer k, face
// index e + (p + 1) k) onto its layer.  The inverted matrices leave
// rounding in the other entries; they are set to their exact value, zero,
// so that the kernel can skip them.  The face order (bottom, top, three
// sides) and a structure that does not hold are reported as errors.
int prism_structure(fr_dvm *h, MixType &T, int p) {
    const int ns = T.ns, nl = p + 1, nt = ns / nl, nft = T.nft;
    if (nt * nl != ns || nft != 2 * nt + 3 * nl * nl)
        return h->fail(FR_DVM_EINVAL, "prism point counts differ from the layered set");
    // the set a face point t lifts onto: column m (end faces) or layer k (sides)
    std::vector<int> col(nft, -1), lay(nft, -1);
    for (int t = 0; t < nft; ++t) {
        const int f = T.ffac[t], i = T.fnode[t];
        if (t < 2 * nt) {
            const int m = t % nt, k = t < nt ? 0 : nl - 1;
            if (f != t / nt || i != m + nt * k) return h->fail(FR_DVM_EINVAL, "prism end-face points out of order");
            col[t] = m;
        } else {
            const int u = t - 2 * nt, k = (u % (nl * nl)) / nl;
            if (f != 2 + u / (nl * nl) || i / nt != k) return h->fail(FR_DVM_EINVAL, "prism side-face points out of order");
            lay[t] = k;
        }
    }
    double dmax = 0.0, lmax = 0.0;
    for (double v : T.D) dmax = std::max(dmax, std::fabs(v));
    for (double v : T.lift) lmax = std::max(lmax, std::fabs(v));
    for (int d = 0; d < 3; ++d)
        for (int i = 0; i < ns; ++i)
            for (int j = 0; j < ns; ++j) {
                double &v = T.D[(d * ns + i) * ns + j];
                const bool couple = d < 2 ? i / nt == j / nt : i % nt == j % nt;
                if (couple) continue;
                if (std::fabs(v) > 1e-9 * dmax) return h->fail(FR_DVM_EINVAL, "prism derivative lacks the layer structure");
                v = 0.0;
            }
    for (int i = 0; i < ns; ++i)
        for (int t = 0; t < nft; ++t) {
            double &v = T.lift[(size_t)t * ns + i];
            const bool onto = col[t] >= 0 ? i % nt == col[t] : i / nt == lay[t];
            if (onto) continue;
            if (std::fabs(v) > 1e-9 * lmax) return h->fail(FR_DVM_EINVAL, "prism lifting lacks the layer structure");
            v = 0.0;
        }
    return FR_DVM_OK;
}

// Reference operators of one element type.
int build_type(fr_dvm *h, MixType &T, int t, int p) {
    T.etype = t;
    const std::vector<V3> x = ref_points(t, p);
    const auto ex = exponents(t, p);
    const int ns = (int)x.size();
    if ((int)ex.size() != ns) return h->fail(FR_DVM_EINVAL, "point set and polynomial space differ");
    T.ns = ns;
    std::vector<double> V(ns * ns), phi(ns), G(ns * 3);
    std::vector<std::array<double, 3>> gr(ns);
    std::vector<double> Vd[3];
    for (int d = 0; d < 3; ++d) Vd[d].assign(ns * ns, 0.0);
    for (int i = 0; i < ns; ++i) {
        basis(ex, p, x[i], phi.data(), reinterpret_cast<double(*)[3]>(gr.data()));
        for (int m = 0; m < ns; ++m) {
            V[i * ns + m] = phi[m];
            for (int d = 0; d < 3; ++d) Vd[d][i * ns + m] = gr[m][d];
        }
    }
    std::vector<double> Vi = V;
    if (!invert(Vi, ns)) return h->fail(FR_DVM_EINVAL, "singular Vandermonde matrix");
    // Lagrange function j at a point with basis values phi: sum_m phi_m Vi[m][j]
    auto lagrange = [&](const V3 &q, std::vector<double> &l) {
        basis(ex, p, q, phi.data(), nullptr);
        l.assign(ns, 0.0);
        for (int m = 0; m < ns; ++m)
            for (int j = 0; j < ns; ++j) l[j] += phi[m] * Vi[m * ns + j];
    };
    T.D.assign(3 * ns * ns, 0.0);
    for (int d = 0; d < 3; ++d)
        for (int i = 0; i < ns; ++i)
            for (int j = 0; j < ns; ++j) {
                double s = 0.0;
                for (int m = 0; m < ns; ++m) s += Vd[d][i * ns + m] * Vi[m * ns + j];
                T.D[(d * ns + i) * ns + j] = s;
            }
    // mass matrix
    std::vector<V3> qx;
    std::vector<double> qw;
    volume_rule(t, p + 3, qx, qw);
    std::vector<double> M(ns * ns, 0.0), l;
    for (size_t q = 0; q < qx.size(); ++q) {
        lagrange(qx[q], l);
        for (int i = 0; i < ns; ++i)
            for (int j = 0; j < ns; ++j) M[i * ns + j] += qw[q] * l[i] * l[j];
    }
    T.W.assign(ns, 0.0);
    for (int i = 0; i < ns; ++i)
        for (int j = 0; j < ns; ++j) T.W[i] += M[i * ns + j];
    std::vector<double> Mi = M;
    if (!invert(Mi, ns)) return h->fail(FR_DVM_EINVAL, "singular mass matrix");
    // faces: points on each, lifting of a unit jump at each
    const std::vector<V3> rv = ref_verts(t);
    T.nface = kNF[t];
    T.fnode.clear();
    T.ffac.clear();
    std::vector<std::vector<double>> cols;
    for (int f = 0; f < T.nface; ++f) {
        const bool quad = kFaceV[t][f][3] >= 0;
        V3 fv[4];
        for (int a = 0; a < (quad ? 4 : 3); ++a) fv[a] = rv[kFaceV[t][f][a]];
        V3 nrm = cross(sub(fv[1], fv[0]), sub(fv[2], fv[0]));
        const double nn = norm(nrm);
        std::vector<int> on;
        for (int i = 0; i < ns; ++i)
            if (std::fabs(dot(sub(x[i], fv[0]), nrm)) < 1e-12 * nn) on.push_back(i);
        std::vector<V3> fx;
        std::vector<double> fw;
        face_rule(fv, quad, p + 3, fx, fw);
        std::vector<double> E(ns * on.size(), 0.0);
        for (size_t q = 0; q < fx.size(); ++q) {
            lagrange(fx[q], l);
            for (int i = 0; i < ns; ++i)
                for (size_t j = 0; j < on.size(); ++j) E[i * on.size() + j] += fw[q] * l[i] * l[on[j]];
        }
        for (size_t j = 0; j < on.size(); ++j) {
            std::vector<double> c(ns, 0.0);
            for (int i = 0; i < ns; ++i)
                for (int k = 0; k < ns; ++k) c[i] += Mi[i * ns + k] * E[k * on.size() + j];
            cols.push_back(c);
            T.fnode.push_back(on[j]);
            T.ffac.push_back(f);
        }
    }
    T.nft = (int)T.fnode.size();
    T.lift.assign((size_t)ns * T.nft, 0.0);
    for (int tt = 0; tt < T.nft; ++tt)
        for (int i = 0; i < ns; ++i) T.lift[(size_t)tt * ns + i] = cols[tt][i];
    return t == FR_DVM_PRISM ? prism_structure(h, T, p) : FR_DVM_OK;
}

template <typename T>
int dalloc(fr_dvm *h, T **p, size_t n) {
    if (hipMalloc(reinterpret_cast<void **>(p), std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        return h->fail(FR_DVM_ENOMEM, "mixed-mesh table allocation failed");
    }
    h->owned_bytes += n * sizeof(T);
    return FR_DVM_OK;
}
template <typename T>
int dput(fr_dvm *h, T **p, const std::vector<T> &v) {
    int rc = dalloc(h, p, v.size());
    if (rc) return rc;
    if (!v.empty() && hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        return h->fail(FR_DVM_EHIP, "mixed-mesh table upload failed");
    return FR_DVM_OK;
}
std::vector<float> to_f32(const std::vector<double> &v) { return std::vector<float>(v.begin(), v.end()); }

}  // namespace

extern "C" int fr_dvm_create_mixed(const fr_dvm_mixed_mesh *mesh, int order, const fr_dvm_vgrid *grid,
                                   fr_dvm_t *out) {
    if (!out) return FR_DVM_EINVAL;
    *out = nullptr;
    if (!mesh || !grid || !mesh->nodes || !mesh->elem_type || !mesh->elem_nodes || !mesh->nbr_elem ||
        !mesh->nbr_face)
        return FR_DVM_EINVAL;
    fr_dvm *h = new fr_dvm();
    auto bail = [&](int rc) { *out = h; return rc; };  // keep the handle so the error is readable
    if (order < 1 || order > kMaxP) return bail(h->fail(FR_DVM_EUNSUPPORTED, "order must be 1..3"));
    if (mesh->n_elem <= 0 || mesh->n_nodes <= 0) return bail(h->fail(FR_DVM_EINVAL, "empty mesh"));
    hipGetDevice(&h->device);
    h->mx = new Mixed();
    Mixed &mx = *h->mx;
    h->p = order;
    h->n = order + 1;
    h->nodes = FR_DVM_NODES_LOBATTO;
    int rc = setup_vgrid(h, grid);
    if (rc) return bail(rc);
    const int64_t ne = mesh->n_elem;
    mx.ne = ne;
    for (int64_t e = 0; e < ne; ++e) {
        const int t = mesh->elem_type[e];
        if (t < 0 || t > 2) return bail(h->fail(FR_DVM_EINVAL, "unknown element type"));
        for (int v = 0; v < kNV[t]; ++v) {
            const int32_t id = mesh->elem_nodes[e * 8 + v];
            if (id < 0 || id >= mesh->n_nodes) return bail(h->fail(FR_DVM_EINVAL, "element node id out of range"));
        }
        mx.t[t].elems.push_back((int32_t)e);
    }
    for (int t = 0; t < 3; ++t)
        if (!mx.t[t].elems.empty() && (rc = build_type(h, mx.t[t], t, order))) return bail(rc);
    // offsets of solution points and face points
    mx.poff.assign(ne + 1, 0);
    mx.toff.assign(ne + 1, 0);
    for (int64_t e = 0; e < ne; ++e) {
        const MixType &T = mx.t[mesh->elem_type[e]];
        mx.poff[e + 1] = mx.poff[e] + T.ns;
        mx.toff[e + 1] = mx.toff[e] + T.nft;
    }
    mx.npts = mx.poff[ne];
    mx.nfp = mx.toff[ne];
    // geometry
    std::vector<double> geo((size_t)ne * kMixGeo, 0.0), wq((size_t)mx.npts);
    std::vector<V3> fpos((size_t)mx.nfp);
    double hmin = 1e300, scale = 0.0;
    for (int64_t i = 0; i < 3 * (int64_t)mesh->n_nodes; ++i) scale = std::max(scale, std::fabs(mesh->nodes[i]));
    for (int64_t e = 0; e < ne; ++e) {
        const int t = mesh->elem_type[e];
        const MixType &T = mx.t[t];
        V3 X[8];
        for (int v = 0; v < kNV[t]; ++v) {
            const double *q = mesh->nodes + 3 * (int64_t)mesh->elem_nodes[e * 8 + v];
            X[v] = {q[0], q[1], q[2]};
        }
        double A[3][3];
        for (int a = 0; a < 3; ++a)
            for (int d = 0; d < 3; ++d) A[d][a] = 0.5 * (X[kAxes[t][a]][d] - X[0][d]);
        for (int v = 0; v < kNV[t]; ++v)
            for (int d = 0; d < 3; ++d) {
                double img = X[0][d];
                for (int a = 0; a < 3; ++a) img += A[d][a] * (kRefV[t][v][a] + 1.0);
                if (std::fabs(img - X[v][d]) > 1e-12 * (1.0 + scale))
                    return bail(h->fail(FR_DVM_EINVAL, "element " + std::to_string(e) + " is not straight (affine)"));
            }
        const double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                           A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                           A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
        if (!(det > 0)) return bail(h->fail(FR_DVM_EINVAL, "element " + std::to_string(e) + ": non-positive Jacobian"));
        double *g = &geo[(size_t)e * kMixGeo];
        // dxi_a/dx_d = (A^-1)[a][d], by cofactors
        g[0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / det;
        g[1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / det;
        g[2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / det;
        g[3] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / det;
        g[4] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / det;
        g[5] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / det;
        g[6] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / det;
        g[7] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / det;
        g[8] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / det;
        V3 cen{0, 0, 0};
        for (int v = 0; v < kNV[t]; ++v)
            for (int d = 0; d < 3; ++d) cen[d] += X[v][d] / kNV[t];
        const std::vector<V3> rv = ref_verts(t);
        double amax = 0.0;
        for (int f = 0; f < T.nface; ++f) {
            const bool quad = kFaceV[t][f][3] >= 0;
            V3 pv[4], qv[4], fc{0, 0, 0};
            const int nv = quad ? 4 : 3;
            for (int a = 0; a < nv; ++a) {
                pv[a] = X[kFaceV[t][f][a]];
                qv[a] = rv[kFaceV[t][f][a]];
                for (int d = 0; d < 3; ++d) fc[d] += pv[a][d] / nv;
            }
            V3 nrm = cross(sub(pv[1], pv[0]), sub(pv[2], pv[0]));
            const double nn = norm(nrm);
            for (int d = 0; d < 3; ++d) nrm[d] /= nn;
            if (dot(nrm, sub(fc, cen)) < 0)
                for (int d = 0; d < 3; ++d) nrm[d] = -nrm[d];
            const double area = face_area(pv, quad);
            amax = std::max(amax, area);
            for (int d = 0; d < 3; ++d) g[9 + 3 * f + d] = nrm[d];
            g[27 + f] = area / face_area(qv, quad) / det;
        }
        double vol = 0.0;
        for (int i = 0; i < T.ns; ++i) {
            wq[mx.poff[e] + i] = T.W[i] * det;
            vol += T.W[i] * det;
        }
        hmin = std::min(hmin, vol / amax);
        // physical positions of the face points
        const std::vector<V3> x = ref_points(t, order);
        for (int tt = 0; tt < T.nft; ++tt) {
            const V3 &r = x[T.fnode[tt]];
            V3 &o = fpos[mx.toff[e] + tt];
            for (int d = 0; d < 3; ++d) o[d] = X[0][d] + A[d][0] * (r[0] + 1) + A[d][1] * (r[1] + 1) + A[d][2] * (r[2] + 1);
        }
    }
    h->hmin = hmin;
    // face-point matching with the neighbours
    std::vector<int64_t> tnb((size_t)mx.nfp, -1);
    const double tol = 1e-9 * (1.0 + scale);
    for (int64_t e = 0; e < ne; ++e) {
        const int t = mesh->elem_type[e];
        const MixType &T = mx.t[t];
        for (int f = 0; f < T.nface; ++f) {
            const int64_t n2 = mesh->nbr_elem[e * 6 + f];
            const int f2 = mesh->nbr_face[e * 6 + f];
            if (n2 < 0 || n2 >= ne) return bail(h->fail(FR_DVM_EINVAL, "mixed meshes need a neighbour across every face"));
            const MixType &T2 = mx.t[mesh->elem_type[n2]];
            if (f2 < 0 || f2 >= T2.nface || mesh->nbr_elem[n2 * 6 + f2] != e || mesh->nbr_face[n2 * 6 + f2] != f)
                return bail(h->fail(FR_DVM_EINVAL, "neighbour relation is not symmetric"));
            std::vector<int64_t> mine, theirs;
            for (int tt = 0; tt < T.nft; ++tt)
                if (T.ffac[tt] == f) mine.push_back(mx.toff[e] + tt);
            for (int tt = 0; tt < T2.nft; ++tt)
                if (T2.ffac[tt] == f2) theirs.push_back(mx.toff[n2] + tt);
            if (mine.size() != theirs.size()) return bail(h->fail(FR_DVM_EINVAL, "neighbouring faces of different shapes"));
            V3 c1{0, 0, 0}, c2{0, 0, 0}, sh;
            for (size_t a = 0; a < mine.size(); ++a)
                for (int d = 0; d < 3; ++d) {
                    c1[d] += fpos[mine[a]][d] / mine.size();
                    c2[d] += fpos[theirs[a]][d] / theirs.size();
                }
            for (int d = 0; d < 3; ++d) {
                const double P = mesh->period[d];
                sh[d] = P > 0 ? P * std::round((c1[d] - c2[d]) / P) : 0.0;
            }
            for (int64_t s : mine) {
                int64_t hit = -1;
                for (int64_t s2 : theirs) {
                    const V3 q = {fpos[s2][0] + sh[0], fpos[s2][1] + sh[1], fpos[s2][2] + sh[2]};
                    if (norm(sub(q, fpos[s])) < tol) {
                        if (hit >= 0) return bail(h->fail(FR_DVM_EINVAL, "coincident face points"));
                        hit = s2;
                    }
                }
                if (hit < 0) return bail(h->fail(FR_DVM_EINVAL, "face points of element " + std::to_string(e) +
                                                                     " face " + std::to_string(f) + " have no match"));
                tnb[s] = hit;
            }
        }
    }
    // the point-wise machinery sees one "element" per solution point
    h->ne = mx.npts;
    h->ns = 1;
    h->nfp = 0;
    h->ncomp = 1;
    if ((rc = finish_create(h, wq))) return bail(rc);
    if ((rc = dput(h, &mx.d_poff, mx.poff)) || (rc = dput(h, &mx.d_toff, mx.toff)) || (rc = dput(h, &mx.d_tnb, tnb)) ||
        (rc = dput(h, &mx.d_geo, geo)) || (rc = dput(h, &mx.d_geof, to_f32(geo))))
        return bail(rc);
    for (int t = 0; t < 3; ++t) {
        MixType &T = mx.t[t];
        if (T.elems.empty()) continue;
        if ((rc = dput(h, &T.d_D, T.D)) || (rc = dput(h, &T.d_lift, T.lift)) || (rc = dput(h, &T.d_Df, to_f32(T.D))) ||
            (rc = dput(h, &T.d_liftf, to_f32(T.lift))) || (rc = dput(h, &T.d_elems, T.elems)) ||
            (rc = dput(h, &T.d_fnode, T.fnode)) || (rc = dput(h, &T.d_ffac, T.ffac)))
            return bail(rc);
    }
    *out = h;
    return FR_DVM_OK;
}

namespace frdvm {

void free_mixed(fr_dvm *h) {
    if (!h->mx) return;
    Mixed &mx = *h->mx;
    void *ptrs[] = {mx.d_poff, mx.d_toff, mx.d_tnb, mx.d_geo, mx.d_geof};
    for (void *p : ptrs)
        if (p) hipFree(p);
    for (MixType &T : mx.t) {
        void *tp[] = {T.d_D, T.d_lift, T.d_Df, T.d_liftf, T.d_elems, T.d_fnode, T.d_ffac};
        for (void *p : tp)
            if (p) hipFree(p);
    }
    delete h->mx;
    h->mx = nullptr;
}

}  // namespace frdvm
