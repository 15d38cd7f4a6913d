// FR residual + collision + Runge-Kutta stage on general hexahedral meshes
// (gfx950): curved 27-node elements, faces met under any orientation,
// farfield and diffuse isothermal wall boundaries.
//
// Paper, Section "Numerical method": per velocity node the transformed flux
// F~_d = (a^d . u) f with the area-scaled contravariant vectors
// a^d = |J| grad xi_d, its divergence along the element's tensor lines, and
// at every flux point the upwind common flux F^I = u_n f- (u_n > 0) or
// u_n f+ (otherwise), u_n = u . n with the area-scaled outward normal; the
// jump F^I - u_n f- enters through the DG-recovering correction.  Exterior
// states (Section "Implementation & problem setup"): the neighbour's trace, the freestream Maxwellian (farfield),
// rho_w M(0, theta_w) (diffuse wall at rest) with rho_w chosen so that no
// mass crosses the wall, or the element's own trace at the mirrored velocity
// (specular symmetry wall).  The collision source (g(Q') - f)/tau and the RK
// combination are those of the box kernel.
//
// Work decomposition: one wave per (element, 64 velocities), one lane per
// velocity; the element's metrics and normals are read through the scalar
// cache, its equilibrium records staged in LDS.  A lane keeps its velocity's
// N^3 values and their residual in a private LDS column; the derivative and
// the face terms are formed line by line, direction by direction.  Every access to f, the
// RK registers and the traces is a run of consecutive velocities.  Traces
// are full (every velocity at every flux point, [e][face][point][k]); a lane
// reads the neighbour trace only where its velocity enters the element.
// The per-point moments are a separate reduction over the velocity axis.
#include <hip/hip_runtime.h>

#include <cstring>

#include "frdvm_common.h"
#include "frdvm_dev.h"

namespace frdvm {

namespace {

constexpr int GMODE_STAGE = 1, GMODE_RESID = 2;
constexpr int kGBlock = 256;  // velocities per workgroup (traces, moments, wall sums)
constexpr int kGWave = 64;    // velocities per workgroup of the stage kernel

template <typename Real>
struct GOps {
    Real D[kMaxN * kMaxN];
    Real lam[2][kMaxN];
    Real corr[2][kMaxN];
};

struct GenArgs {
    GOps<float> of;
    GOps<double> od;
    VGrid vg;
    int nu, nut, ncomp;  // velocities; state values per point (ncomp components of nu)
    int nvb, nvw;        // blocks of 256 and of 64 state values per element
    double gwall;        // the pair's G wall factor delta theta_w / 2
    const double *gfp;   // [npts] the pair's G equilibrium factor delta theta / 2
    const double *wax;   // [3][64] 1-D trapezoid weights
    const double *wJ;    // [ne][ns] Gauss weight x |J| (positivity limiter)
    const double *S;     // [ne][ns][3][3]
    const double *ijac;  // [ne][ns]
    const double *nf;    // [ne][6][nfp][3]
    const float *Sf, *ijacf, *nff;  // the same in FP32
    const int32_t *conn; // [ne][6][4]
    const int32_t *wall; // [nwall]
    double *rw;          // [ne*6][nfp]
    const double *mw;    // [nu]
    const double *finf;  // [nu]
    StageArgs sa;
    int do_traces;
};

template <typename Real>
__device__ __forceinline__ const GOps<Real> &gops(const GenArgs &A);
template <>
__device__ __forceinline__ const GOps<float> &gops<float>(const GenArgs &A) { return A.of; }
template <>
__device__ __forceinline__ const GOps<double> &gops<double>(const GenArgs &A) { return A.od; }

// Metric tables in the working precision, read through the scalar cache
// (the indices are uniform over the workgroup).
template <typename Real>
using cptr = const __attribute__((address_space(4))) Real *;
template <typename Real>
struct Metrics {
    cptr<Real> S, ijac, nf;
};
__device__ __forceinline__ Metrics<float> metrics(const GenArgs &A, float) {
    return {(cptr<float>)A.Sf, (cptr<float>)A.ijacf, (cptr<float>)A.nff};
}
__device__ __forceinline__ Metrics<double> metrics(const GenArgs &A, double) {
    return {(cptr<double>)A.S, (cptr<double>)A.ijac, (cptr<double>)A.nf};
}

template <typename Real>
__device__ __forceinline__ Real gexp(double E);
template <>
__device__ __forceinline__ float gexp<float>(double E) { return exp_to_f32(E); }
template <>
__device__ __forceinline__ double gexp<double>(double E) { return exp(E); }

// Uniform base + the lane's byte offset (a run of consecutive velocities).
template <typename T>
__device__ __forceinline__ T ldo(const T *base, uint32_t boff) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + boff);
}
template <typename T>
__device__ __forceinline__ void sto(T *base, uint32_t boff, T v) {
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + boff) = v;
}

// Velocity node umin + i du (two roundings, as on the host).
__device__ __forceinline__ double node_u(const VGrid &vg, int d, int i) {
    return __dadd_rn(vg.umin[d], __dmul_rn((double)i, vg.du[d]));
}

// Velocity node k = i + n0 (j + n1 l) -> (i, j, l).  The quotients are taken
// in FP32 from (k + 1/2) times the reciprocal, exact for k < 2^22 (a grid
// has at most 64^3 nodes), instead of integer divisions.
__device__ __forceinline__ void split_k(const VGrid &vg, int k, int iv[3]) {
    const int n0 = vg.nv[0], n01 = vg.nv[0] * vg.nv[1];
    const int q2 = (int)(((float)k + 0.5f) * (1.0f / (float)n01));
    const int r = k - q2 * n01;
    const int q1 = (int)(((float)r + 0.5f) * (1.0f / (float)n0));
    iv[0] = r - q1 * n0;
    iv[1] = q1;
    iv[2] = q2;
}

template <int N>
__device__ __forceinline__ constexpr int spt(int i, int j, int l) { return i + N * (j + N * l); }

// m-th point of the line along axis d through face point (a, b); (a, b) run
// along the two other axes in increasing order.
template <int N>
__device__ __forceinline__ constexpr int line_pt(int d, int a, int b, int m) {
    return d == 0 ? spt<N>(m, a, b) : (d == 1 ? spt<N>(a, m, b) : spt<N>(a, b, m));
}

// Own face point (a, b) -> neighbour face point under orientation code o.
template <int N>
__device__ __forceinline__ int nbr_point(int o, int a, int b) {
    int x = (o & 1) ? b : a, y = (o & 1) ? a : b;
    if (o & 2) x = N - 1 - x;
    if (o & 4) y = N - 1 - y;
    return x + N * y;
}

// Traces of f at every flux point of the element, every velocity.
template <typename Real, int P>
__global__ __launch_bounds__(kGBlock) void k_gen_traces(const GenArgs A, const Real *__restrict__ f,
                                                         Real *__restrict__ tr) {
    constexpr int N = P + 1, NS = N * N * N, NFP = N * N;
    const int64_t e = blockIdx.x / A.nvb;
    const int k = (int)(blockIdx.x % A.nvb) * kGBlock + threadIdx.x;
    if (k >= A.nut) return;
    const int64_t nu = A.nut;  // stride of a solution point
    const GOps<Real> &op = gops<Real>(A);
    const uint32_t ko = (uint32_t)k * (uint32_t)sizeof(Real);
    const Real *fe = f + e * NS * nu;
    Real v[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) v[s] = ldo(fe + s * nu, ko);
    Real *te = tr + e * 6 * NFP * nu;
#pragma unroll
    for (int face = 0; face < 6; ++face) {
        const int d = face / 2, side = face & 1;
#pragma unroll
        for (int b = 0; b < N; ++b)
#pragma unroll
            for (int a = 0; a < N; ++a) {
                Real t = Real(0);
#pragma unroll
                for (int m = 0; m < N; ++m) t += op.lam[side][m] * v[line_pt<N>(d, a, b, m)];
                sto(te + (face * NFP + a + N * b) * nu, ko, t);
            }
    }
}

// Moments of one solution point over the velocity grid (FP64, fixed order),
// one wave per point and kMomPts points per workgroup.  Lane t of the wave
// takes the (x, y) nodes t, t + 64, ... and walks each one's z column: the
// nodes of a z step are consecutive over the lanes (coalesced), and along
// the column only the z weight and u_z vary, so the column is summed as
// (sum w_z f, sum w_z u_z f, sum w_z u_z^2 f): three multiply-adds per value
// with wave-uniform coefficients; the (x, y) weight and velocity close the
// column into the moments, and a wave butterfly sums the lanes.  (A
// workgroup per point, its threads over the columns, spent most of its time
// starting workgroups and reducing across waves.)  BGK: rho, rho U, E; ES:
// rho, rho U and the raw second moments xx yy zz xy xz yz; the pair's G adds
// its integral (last slot).
constexpr int kMomMaxZ = 64;
constexpr int kMomPts = 4;  // points (waves) per workgroup
template <typename Real, int NMOM>
__global__ __launch_bounds__(64 * kMomPts) void k_gen_moments(const GenArgs A, const Real *__restrict__ f,
                                                              double *__restrict__ Q, int64_t npts) {
    constexpr bool PAIR = NMOM == 6 || NMOM == 11;
    __shared__ double tz[kMomMaxZ][3];  // w_z, w_z u_z, w_z u_z^2
    const int nx = A.vg.nv[0], ny = A.vg.nv[1], nz = A.vg.nv[2], nxy = nx * ny;
    for (int iz = threadIdx.x; iz < nz; iz += blockDim.x) {
        const double w = A.wax[128 + iz], u = node_u(A.vg, 2, iz);
        tz[iz][0] = w;
        tz[iz][1] = w * u;
        tz[iz][2] = (w * u) * u;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t pt = (int64_t)blockIdx.x * kMomPts + (threadIdx.x >> 6);
    if (pt >= npts) return;  // (no barrier follows)
    const Real *fp = f + pt * A.nut;
    double M[NMOM];
#pragma unroll
    for (int a = 0; a < NMOM; ++a) M[a] = 0.0;
    for (int t = lane; t < nxy; t += 64) {
        const int iy = t / nx, ix = t - iy * nx;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, g0 = 0.0;
#pragma unroll 4
        for (int iz = 0; iz < nz; ++iz) {
            const double x = (double)fp[t + iz * nxy];
            s0 = fma(tz[iz][0], x, s0);
            s1 = fma(tz[iz][1], x, s1);
            s2 = fma(tz[iz][2], x, s2);
            if constexpr (PAIR) g0 = fma(tz[iz][0], (double)fp[A.nu + t + iz * nxy], g0);
        }
        const double W = A.wax[ix] * A.wax[64 + iy];
        const double ux = node_u(A.vg, 0, ix), uy = node_u(A.vg, 1, iy);
        const double a0 = W * s0, a1 = W * s1, a2 = W * s2;
        M[0] += a0;
        M[1] = fma(ux, a0, M[1]);
        M[2] = fma(uy, a0, M[2]);
        M[3] += a1;
        if constexpr (NMOM == 5 || NMOM == 6) {
            M[4] = fma(0.5, fma(ux * ux + uy * uy, a0, a2), M[4]);
        } else {
            M[4] = fma(ux * ux, a0, M[4]);
            M[5] = fma(uy * uy, a0, M[5]);
            M[6] += a2;
            M[7] = fma(ux * uy, a0, M[7]);
            M[8] = fma(ux, a1, M[8]);
            M[9] = fma(uy, a1, M[9]);
        }
        if constexpr (PAIR) M[NMOM - 1] = fma(W, g0, M[NMOM - 1]);
    }
#pragma unroll
    for (int a = 0; a < NMOM; ++a) {
        double v = M[a];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
        if (lane == a) Q[pt * NMOM + a] = v;
    }
}
inline unsigned gen_moment_grid(int64_t npts) { return (unsigned)((npts + kMomPts - 1) / kMomPts); }

// Wall density at each flux point of the diffuse-wall faces: the outflow
// mass flux of the interior trace over the inflow flux of the unit wall
// Maxwellian, rho_w = sum_{u_n>0} w u_n f- / sum_{u_n<0} w |u_n| M_w.
template <typename Real, int P>
__global__ __launch_bounds__(kGBlock) void k_gen_wall(const GenArgs A, const Real *__restrict__ tr) {
    constexpr int N = P + 1, NFP = N * N;
    __shared__ double red[kGBlock / 64][2];
    const int64_t fid = A.wall[blockIdx.x / NFP];
    const int fp = blockIdx.x % NFP;
    const double *nv = A.nf + (fid * NFP + fp) * 3;
    const double n0 = nv[0], n1 = nv[1], n2 = nv[2];
    const Real *t = tr + (fid * NFP + fp) * (int64_t)A.nut;  // F part of the trace
    double out = 0.0, in = 0.0;
    for (int k = threadIdx.x; k < A.nu; k += kGBlock) {
        int iv[3];
        split_k(A.vg, k, iv);
        const double w = A.wax[iv[0]] * A.wax[64 + iv[1]] * A.wax[128 + iv[2]];
        const double un = node_u(A.vg, 0, iv[0]) * n0 + node_u(A.vg, 1, iv[1]) * n1 + node_u(A.vg, 2, iv[2]) * n2;
        if (un > 0.0)
            out += w * un * (double)t[k];
        else
            in -= w * un * A.mw[k];
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        out += __shfl_xor(out, o);
        in += __shfl_xor(in, o);
    }
    if (lane == 0) {
        red[wv][0] = out;
        red[wv][1] = in;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double so = red[0][0], si = red[0][1];
#pragma unroll
        for (int q = 1; q < kGBlock / 64; ++q) {
            so += red[q][0];
            si += red[q][1];
        }
        A.rw[fid * NFP + fp] = si > 0.0 ? so / si : 0.0;
    }
}

// One wave per (element, 64 velocities).  Each lane keeps its velocity's N^3
// residual accumulators in its own LDS column (lane-private: no barrier
// between the phases), and its N^3 stage values in registers (p <= 2: the
// loops over directions, lines and flux points unrolled, so every value has
// a fixed register; the LDS left per wave admits 3 (FP32) / 2 (FP64) waves
// per SIMD, which the register target matches) or in a second LDS column
// (p = 3: loops rolled, the registers holding only the current line).  (With the accumulators in
// registers and the direction loop unrolled, p = 2 needs 175 VGPRs in FP32
// and p = 3 all 256 with scratch: no occupancy is gained.)
template <typename Real, int P>
constexpr bool gen_freg() {
    return P <= 2;
}
template <typename Real, int P, int MODE>
__global__ __launch_bounds__(kGWave) __attribute__((amdgpu_waves_per_eu(gen_freg<Real, P>() ? (sizeof(Real) == 4 ? 3 : 2) : 1))) void
k_gen_stage(const GenArgs A) {
    constexpr int N = P + 1, NS = N * N * N, NFP = N * N;
    constexpr bool STAGE = MODE == GMODE_STAGE;
    constexpr int CHF = NS <= 27 ? NS : 2 * NFP;  // values requested together
    constexpr bool FREG = gen_freg<Real, P>();
    constexpr bool EARLY_X = STAGE && NS <= 27 && !FREG;
    constexpr int UNR = FREG ? 64 : 1;  // unroll of the loops that index the stage values
    __shared__ Real sf[FREG ? 1 : NS][kGWave];
    Real fv[FREG ? NS : 1];
    // the lane's stage value at point s (s a compile-time index where FREG)
    auto F = [&](int s) -> Real & {
        if constexpr (FREG) return fv[s];
        else return sf[s][threadIdx.x];
    };
    __shared__ Real sa[NS][kGWave];
    __shared__ double sEb[STAGE ? NS * 8 : 1];
    __shared__ double sEv[STAGE ? NS * 3 : 1];
    __shared__ double sLg[STAGE ? NS : 1];  // log of the pair's G factor per point
    const int64_t e = blockIdx.x / A.nvw;
    const int lane = threadIdx.x;
    const int k = (int)(blockIdx.x % A.nvw) * kGWave + lane;
    const bool collide = STAGE && A.sa.collide;
    if (collide) {
        for (int s = lane; s < NS; s += kGWave) {
            const double *q = A.sa.eq + (e * NS + s) * kEqW;
            double *b = &sEb[s * 8];
            b[0] = -0.5 * q[EQ_B];
            b[1] = -0.5 * q[EQ_B + 1];
            b[2] = -0.5 * q[EQ_B + 2];
            b[3] = -q[EQ_B + 3];
            b[4] = -q[EQ_B + 4];
            b[5] = -q[EQ_B + 5];
            b[6] = q[EQ_C0];
            b[7] = q[EQ_INVTAU];
            sEv[s * 3] = q[EQ_V];
            sEv[s * 3 + 1] = q[EQ_V + 1];
            sEv[s * 3 + 2] = q[EQ_V + 2];
            const double gf = A.ncomp == 2 ? A.gfp[e * NS + s] : 1.0;
            sLg[s] = gf > 0.0 ? log(gf) : -1000.0;
        }
    }
    __syncthreads();
    if (k >= A.nut) return;

    const GOps<Real> &op = gops<Real>(A);
    const Metrics<Real> G = metrics(A, Real(0));
    const cptr<Real> gS = G.S + e * NS * 9, gJ = G.ijac + e * NS, gN = G.nf + e * 6 * NFP * 3;
    const int64_t nu = A.nut;  // stride of a solution point
    const int comp = k >= A.nu, kv = k - comp * A.nu;  // component, velocity node
    int iv[3];
    split_k(A.vg, kv, iv);
    const double ud[3] = {node_u(A.vg, 0, iv[0]), node_u(A.vg, 1, iv[1]), node_u(A.vg, 2, iv[2])};
    const Real u0 = (Real)ud[0], u1 = (Real)ud[1], u2 = (Real)ud[2];
    const int64_t eoff = e * NS * nu;
    const uint32_t ko = (uint32_t)k * (uint32_t)sizeof(Real), k8 = (uint32_t)k * 8u, kv8 = (uint32_t)kv * 8u;
    const Real *fe = reinterpret_cast<const Real *>(A.sa.f) + eoff;
    // all of f (two layers at a time at p = 3) requested together
#pragma unroll 1
    for (int s0 = 0; s0 < NS; s0 += CHF) {
        Real v[CHF];
#pragma unroll
        for (int r = 0; r < CHF; ++r) v[r] = ldo(fe + (s0 + r) * nu, ko);
#pragma unroll
        for (int r = 0; r < CHF; ++r) F(s0 + r) = v[r];
    }
    // the second RK register of the stage, requested now (p <= 2) so that
    // the FR work covers its latency
    const bool useX = STAGE && (A.sa.scheme == 0 ? A.sa.alpha != 0.0 : A.sa.lsA != 0.0);
    const Real *XE = (A.sa.scheme == 0 ? reinterpret_cast<const Real *>(A.sa.fn) : reinterpret_cast<const Real *>(A.sa.dF)) + eoff;
    Real xe[EARLY_X ? NS : 1];
    if constexpr (EARLY_X) {
#pragma unroll
        for (int s = 0; s < NS; ++s) xe[s] = useX ? ldo(XE + s * nu, ko) : Real(0);
    }
    // Divergence and interface corrections, direction by direction: along
    // each line of direction d the transformed flux F_d = (a^d . u) f, its
    // derivative, and the corrections of the line's two flux points on the
    // faces 2d and 2d+1 are formed in registers; each point's accumulator
    // is then written once per direction (the first direction initialises
    // it), so no accumulator waits on another update of itself.
    const Real *tin = reinterpret_cast<const Real *>(A.sa.tr_in);
#pragma unroll UNR
    for (int d = 0; d < 3; ++d) {
        if constexpr (FREG) {
            // one direction's exterior values in registers at a time
            asm volatile("" ::: "memory");
            __builtin_amdgcn_sched_barrier(0);
        }
        // the exterior values of both faces of the axis, requested together
        Real un[2][NFP], ext[2][NFP];
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int face = 2 * d + side;
            const int32_t *c = A.conn + (e * 6 + face) * 4;
            const int32_t nb = c[0], nface = c[1], orient = c[2], bc = c[3];
            const cptr<Real> nv = gN + face * NFP * 3;
#pragma unroll
            for (int q = 0; q < NFP; ++q)
                un[side][q] = nv[3 * q] * u0 + nv[3 * q + 1] * u1 + nv[3 * q + 2] * u2;
            if (nb >= 0) {
                const Real *tn = tin + ((int64_t)nb * 6 + nface) * NFP * nu;
#pragma unroll
                for (int q = 0; q < NFP; ++q)
                    ext[side][q] =
                        un[side][q] < Real(0) ? ldo(tn + nbr_point<N>(orient, q % N, q / N) * nu, ko) : Real(0);
            } else if (bc == 1) {
                const Real fi = (Real)ldo(A.finf, k8);
#pragma unroll
                for (int q = 0; q < NFP; ++q) ext[side][q] = fi;
            } else if (bc == 3) {
                // specular: the own trace at the velocity mirrored in the
                // face's axis (orient holds the axis)
                const int str = orient == 0 ? 1 : (orient == 1 ? A.vg.nv[0] : A.vg.nv[0] * A.vg.nv[1]);
                const int ia = orient == 0 ? iv[0] : (orient == 1 ? iv[1] : iv[2]);
                const int km = k + (A.vg.nv[orient] - 1 - 2 * ia) * str;  // same component
                const uint32_t kmo = (uint32_t)km * (uint32_t)sizeof(Real);
                const Real *to = tin + (e * 6 + face) * NFP * nu;
#pragma unroll
                for (int q = 0; q < NFP; ++q) ext[side][q] = un[side][q] < Real(0) ? ldo(to + q * nu, kmo) : Real(0);
            } else {
                const double mw = ldo(A.mw, kv8) * (comp ? A.gwall : 1.0);
#pragma unroll
                for (int q = 0; q < NFP; ++q) ext[side][q] = (Real)(A.rw[(e * 6 + face) * NFP + q] * mw);
            }
        }
#pragma unroll
        for (int q = 0; q < NFP; ++q) {
            const int a = q % N, b = q / N;
            int pts[N];
            Real fl[N], Fd[N];
#pragma unroll
            for (int m = 0; m < N; ++m) {
                pts[m] = line_pt<N>(d, a, b, m);
                fl[m] = F(pts[m]);
                const cptr<Real> Sm = gS + pts[m] * 9 + 3 * d;
                Fd[m] = (Sm[0] * u0 + Sm[1] * u1 + Sm[2] * u2) * fl[m];
            }
            Real acc[N];
#pragma unroll
            for (int r = 0; r < N; ++r) {
                Real t = Real(0);
#pragma unroll
                for (int m = 0; m < N; ++m) t += op.D[r * N + m] * Fd[m];
                acc[r] = t;
            }
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                if (un[side][q] < Real(0)) {
                    Real fm = Real(0);
#pragma unroll
                    for (int m = 0; m < N; ++m) fm += op.lam[side][m] * fl[m];
                    const Real jump = un[side][q] * (ext[side][q] - fm);
#pragma unroll
                    for (int r = 0; r < N; ++r) acc[r] += op.corr[side][r] * jump;
                }
            }
#pragma unroll
            for (int r = 0; r < N; ++r) sa[pts[r]][lane] = d == 0 ? acc[r] : sa[pts[r]][lane] + acc[r];
        }
    }
    if (MODE == GMODE_RESID) {
        Real *R = reinterpret_cast<Real *>(A.sa.fout) + eoff;
#pragma unroll 4
        for (int s = 0; s < NS; ++s) sto(R + s * nu, ko, -sa[s][lane] * gJ[s]);
        return;
    }
    // collision source and the Runge-Kutta combination
    const Real dt = (Real)A.sa.dt;
    Real *outE = reinterpret_cast<Real *>(A.sa.fout) + eoff;
    Real *dFE = reinterpret_cast<Real *>(A.sa.dF) + eoff;
    // positivity limiter: the result is held in the lane's column until its
    // element mean and smallest value are known
    const bool limit = A.sa.positivity != 0;
    const cptr<double> gW = (cptr<double>)A.wJ + e * NS;
    double lim_int = 0.0, lim_w = 0.0;
    Real lim_min = Real(0);
#pragma unroll
    for (int s0 = 0; s0 < NS; s0 += NFP) {
        // (p = 3) the layer's second-register values requested together
        Real xv[NFP];
#pragma unroll
        for (int r = 0; r < NFP; ++r)
            xv[r] = EARLY_X ? xe[EARLY_X ? s0 + r : 0] : (useX ? ldo(XE + (s0 + r) * nu, ko) : Real(0));
#pragma unroll
        for (int r = 0; r < NFP; ++r) {
            const int s = s0 + r;
            const Real fq = F(s);
            Real L = -sa[s][lane] * gJ[s];
            if (collide) {
                const double *bq = &sEb[s * 8];
                const double c0 = ud[0] - sEv[s * 3], c1 = ud[1] - sEv[s * 3 + 1], c2 = ud[2] - sEv[s * 3 + 2];
                double t0 = bq[0] * c0;
                t0 = fma(bq[3], c1, t0);
                t0 = fma(bq[4], c2, t0);
                double t1 = bq[1] * c1;
                t1 = fma(bq[5], c2, t1);
                const double t2 = bq[2] * c2;
                double E = fma(c0, t0, comp ? bq[6] + sLg[s] : bq[6]);
                E = fma(c1, t1, E);
                E = fma(c2, t2, E);
                L += (gexp<Real>(E) - fq) * (Real)bq[7];
            }
            // the result, in FP64 for the stochastic rounding of the FP32 state
            double fod;
            if (A.sa.scheme == 0) {
                fod = A.sa.beta * ((double)fq + (double)(dt * L));
                if (useX) fod = fma(A.sa.alpha, (double)xv[r], fod);
            } else {
                Real dd = dt * L;
                if (useX) dd += (Real)A.sa.lsA * xv[r];
                if (A.sa.keep_dF) sto(dFE + s * nu, ko, dd);
                fod = fma(A.sa.lsB, (double)dd, (double)fq);
            }
            Real fo;
            if constexpr (sizeof(Real) == 4)
                fo = round_stochastic(fod, round_bits(A.sa.seed, (uint32_t)(e * NS + s), (uint32_t)k));
            else
                fo = (Real)fod;
            F(s) = fo;
            sto(outE + s * nu, ko, fo);
            if constexpr (FREG) {
                // two points' chains in flight at a time
                if (r % 2 == 1) {
                    asm volatile("" ::: "memory");
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        }
    }
    if (limit) {
        // the result's element integral and smallest value at the solution points
#pragma unroll UNR
        for (int s = 0; s < NS; ++s) {
            Real fo = F(s);
            asm volatile("" : "+v"(fo));  // (converted here, not kept in FP64 from the stage loop)
            lim_int = fma(gW[s], (double)fo, lim_int);
            lim_w += gW[s];
            lim_min = s == 0 ? fo : (fo < lim_min ? fo : lim_min);
        }
    }
    // Traces of the result at every flux point; with the positivity limiter
    // the same pass finds the smallest value of the element polynomial at its
    // solution and flux points.  Where that is negative (rare: f is positive
    // almost everywhere) the lane scales its polynomial about the element mean
    // (weights Gauss x |J|), so that the smallest value becomes zero and the
    // element integral of the value, hence every moment, is kept, and stores
    // the values and traces again.
    Real *te = reinterpret_cast<Real *>(A.sa.tr_out) + e * 6 * NFP * nu;
    auto trace_pass = [&](bool store, bool find_min) {
#pragma unroll UNR
        for (int face = 0; face < 6; ++face) {
            const int d = face / 2, side = face & 1;
            if constexpr (FREG) {
                // one face's traces in registers at a time
                asm volatile("" ::: "memory");
                __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll UNR
            for (int q = 0; q < NFP; ++q) {
                const int a = q % N, b = q / N;
                Real t = Real(0);
#pragma unroll
                for (int m = 0; m < N; ++m) t += op.lam[side][m] * F(line_pt<N>(d, a, b, m));
                if (store) sto(te + (face * NFP + q) * nu, ko, t);
                if (find_min) lim_min = t < lim_min ? t : lim_min;
            }
        }
    };
    if (A.do_traces || limit) trace_pass(A.do_traces, limit);
    if (limit && lim_min < Real(0)) {
        const double mean = lim_int / lim_w;
        const double th = mean > 0.0 ? mean / (mean - (double)lim_min) : 0.0;
#pragma unroll UNR
        for (int s = 0; s < NS; ++s) {
            const Real v = (Real)fma(th, (double)F(s) - mean, mean);
            F(s) = v;
            sto(outE + s * nu, ko, v);
        }
        if (A.do_traces) trace_pass(true, false);
    }
}

int gcheck(fr_dvm *h, const char *what) {
    hipError_t st = hipGetLastError();
    if (st != hipSuccess) return h->fail(FR_DVM_EHIP, std::string(what) + ": " + hipGetErrorString(st));
    return FR_DVM_OK;
}

template <typename Real, int P>
int gen_run(fr_dvm *h, int mode, const GenArgs &A, int do_moments) {
    const unsigned blocks = (unsigned)(h->ne * A.nvb);
    const int64_t npts = h->ne * h->ns;
    auto moments = [&](const void *src) {
        const Real *fs = reinterpret_cast<const Real *>(src);
        switch (h->nmom) {
            case 5: hipLaunchKernelGGL((k_gen_moments<Real, 5>), dim3(gen_moment_grid(npts)), dim3(64 * kMomPts), 0, h->stream, A, fs, A.sa.Q, (int64_t)npts); break;
            case 6: hipLaunchKernelGGL((k_gen_moments<Real, 6>), dim3(gen_moment_grid(npts)), dim3(64 * kMomPts), 0, h->stream, A, fs, A.sa.Q, (int64_t)npts); break;
            case 10: hipLaunchKernelGGL((k_gen_moments<Real, 10>), dim3(gen_moment_grid(npts)), dim3(64 * kMomPts), 0, h->stream, A, fs, A.sa.Q, (int64_t)npts); break;
            default: hipLaunchKernelGGL((k_gen_moments<Real, 11>), dim3(gen_moment_grid(npts)), dim3(64 * kMomPts), 0, h->stream, A, fs, A.sa.Q, (int64_t)npts);
        }
        return gcheck(h, "moment kernel");
    };
    int rc;
    if (mode == 0) {
        if (A.do_traces) {
            hipLaunchKernelGGL((k_gen_traces<Real, P>), dim3(blocks), dim3(kGBlock), 0, h->stream, A,
                               reinterpret_cast<const Real *>(A.sa.f), reinterpret_cast<Real *>(A.sa.tr_out));
            if ((rc = gcheck(h, "trace kernel"))) return rc;
        }
        return do_moments ? moments(A.sa.f) : FR_DVM_OK;
    }
    if (h->nwall) {
        hipLaunchKernelGGL((k_gen_wall<Real, P>), dim3((unsigned)(h->nwall * h->nfp)), dim3(kGBlock), 0, h->stream,
                           A, reinterpret_cast<const Real *>(A.sa.tr_in));
        if ((rc = gcheck(h, "wall kernel"))) return rc;
    }
    const unsigned wblocks = (unsigned)(h->ne * A.nvw);
    if (mode == GMODE_RESID)
        hipLaunchKernelGGL((k_gen_stage<Real, P, GMODE_RESID>), dim3(wblocks), dim3(kGWave), 0, h->stream, A);
    else
        hipLaunchKernelGGL((k_gen_stage<Real, P, GMODE_STAGE>), dim3(wblocks), dim3(kGWave), 0, h->stream, A);
    if ((rc = gcheck(h, "general stage kernel"))) return rc;
    return (mode == GMODE_STAGE && do_moments) ? moments(A.sa.fout) : FR_DVM_OK;
}

template <typename Real>
int gen_p(fr_dvm *h, int mode, const GenArgs &A, int do_moments) {
    switch (h->p) {
        case 1: return gen_run<Real, 1>(h, mode, A, do_moments);
        case 2: return gen_run<Real, 2>(h, mode, A, do_moments);
        case 3: return gen_run<Real, 3>(h, mode, A, do_moments);
    }
    return h->fail(FR_DVM_EUNSUPPORTED, "order");
}

// ---- mixed meshes of straight hexahedra, prisms and tetrahedra ----
//
// Nodal FR with the DG-recovering correction on each element (Section
// "Numerical method"): with f the element's values at its solution points,
//   R_i = -sum_j (sum_a c_a D_a[i][j]) f_j
//         - sum_t lift[i][t] s_f min(u.n_f, 0) (f_nb,t - f_node(t)),
// c_a = u . grad xi_a (constant on a straight element), t running over the
// face points (the solution points on each face, faces in order), f_nb,t the
// neighbour's trace at the same position, s_f = |J_face| / |J|.  One wave per
// (element, 64 velocities), one lane per velocity, the values and residuals
// of the lane in LDS columns, the operators read through the scalar cache.
// The collision source and the RK combination are those of the hexahedral
// kernels; the result's traces are its values at the face points.
struct MixArgs {
    VGrid vg;
    int nu, nvw;
    const int32_t *elems;                 // elements of the launched type
    const int64_t *poff, *toff, *tnb;     // first point / face point of each element; neighbour face point
    const double *geo;                    // [ne][kMixGeo]
    const float *geof;
    const double *D, *lift;               // the type's operators: D [3][ns][ns], lift [nft][ns]
    const float *Df, *liftf;
    const int32_t *fnode, *ffac;          // [nft] solution point and face of each face point
    StageArgs sa;
    int do_traces;
};

template <typename Real>
struct MixOps {
    cptr<Real> geo, D, lift;
};
__device__ __forceinline__ MixOps<float> mix_ops(const MixArgs &A, float) {
    return {(cptr<float>)A.geof, (cptr<float>)A.Df, (cptr<float>)A.liftf};
}
__device__ __forceinline__ MixOps<double> mix_ops(const MixArgs &A, double) {
    return {(cptr<double>)A.geo, (cptr<double>)A.D, (cptr<double>)A.lift};
}

// PL: Gauss-Lobatto layers of a prism (0: other element types).  A prism's
// in-plane derivative operators couple only the points of one layer and its
// axial one only those of one column, an end-face point lifts onto its
// column and a side-face point onto its layer (the host stores the other
// entries as exact zeros and checks the face order): the volume term reads
// 2 NS (NS / PL) + NS PL operator entries instead of 3 NS^2 and the faces
// 2 NS + 3 PL NS instead of NS NFT, in the order of the dense sums.
template <typename Real, int NS, int NFT, int MODE, int PL>
__global__ __launch_bounds__(kGWave) void k_mix_stage(const MixArgs A) {
    // up to 40 points (tetrahedra, prisms, hexahedra to p = 2) a lane keeps
    // its values and residuals in registers and the dense products run fully
    // unrolled with the operator entries as scalar operands; above, both sit
    // in LDS columns
    constexpr bool REG = NS <= 40;
    __shared__ Real sf[NS][kGWave];
    __shared__ Real sa[REG ? 1 : NS][kGWave];
    const int64_t e = A.elems[blockIdx.x / A.nvw];
    const int lane = threadIdx.x;
    const int k = (int)(blockIdx.x % A.nvw) * kGWave + lane;
    const bool act = k < A.nu;
    const int kk = act ? k : 0;  // an idle lane works on node 0 and stores nothing
    const int64_t nu = A.nu;
    const uint32_t ko = (uint32_t)kk * (uint32_t)sizeof(Real);
    const int64_t p0 = A.poff[e], t0 = A.toff[e];
    const MixOps<Real> op = mix_ops(A, Real(0));
    const cptr<Real> g = op.geo + e * kMixGeo;
    const cptr<int32_t> fnode = (cptr<int32_t>)A.fnode, ffac = (cptr<int32_t>)A.ffac;
    int iv[3];
    split_k(A.vg, kk, iv);
    const double ud[3] = {node_u(A.vg, 0, iv[0]), node_u(A.vg, 1, iv[1]), node_u(A.vg, 2, iv[2])};
    const Real u0 = (Real)ud[0], u1 = (Real)ud[1], u2 = (Real)ud[2];
    Real c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) c[a] = u0 * g[3 * a] + u1 * g[3 * a + 1] + u2 * g[3 * a + 2];
    const Real *fE = reinterpret_cast<const Real *>(A.sa.f) + p0 * nu;
    const Real *trI = reinterpret_cast<const Real *>(A.sa.tr_in);
    // the upwind jump at face point t, scaled (0 where the velocity leaves)
    auto jump_at = [&](int t) {
        const int f = ffac[t];
        const Real un = u0 * g[9 + 3 * f] + u1 * g[10 + 3 * f] + u2 * g[11 + 3 * f];
        Real jump = Real(0);
        if (un < Real(0)) jump = un * g[27 + f] * (ldo(trI + A.tnb[t0 + t] * nu, ko) - sf[fnode[t]][lane]);
        return jump;
    };
    Real fv[REG ? NS : 1], r[REG ? NS : 1];
    if constexpr (REG) {
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            fv[i] = ldo(fE + i * nu, ko);
            sf[i][lane] = fv[i];
            r[i] = Real(0);
        }
        // volume: r_i = -sum_a c_a (D_a f)_i
#pragma unroll
        for (int a = 0; a < 3; ++a) {
#pragma unroll
            for (int i = 0; i < NS; ++i) {
                Real gi = Real(0);
                if constexpr (PL > 0) {
                    constexpr int NT = NS / PL;  // points per layer
                    if (a < 2) {
                        const int j0 = i / NT * NT;  // the layer of point i
#pragma unroll
                        for (int m = 0; m < NT; ++m) gi = fma(op.D[(a * NS + i) * NS + j0 + m], fv[j0 + m], gi);
                    } else {
                        const int m0 = i % NT;  // the column of point i
#pragma unroll
                        for (int k = 0; k < PL; ++k) gi = fma(op.D[(a * NS + i) * NS + m0 + NT * k], fv[m0 + NT * k], gi);
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < NS; ++j) gi = fma(op.D[(a * NS + i) * NS + j], fv[j], gi);
                }
                r[i] = fma(-c[a], gi, r[i]);
            }
        }
        // faces
        if constexpr (PL > 0) {
            constexpr int NT = NS / PL;
            // bottom and top faces: face point m lifts onto column m
#pragma unroll 1
            for (int f = 0; f < 2; ++f) {
#pragma unroll
                for (int m = 0; m < NT; ++m) {
                    const int t = f * NT + m;
                    const Real jump = jump_at(t);
#pragma unroll
                    for (int k = 0; k < PL; ++k) {
                        const int i = m + NT * k;
                        r[i] = fma(-op.lift[t * NS + i], jump, r[i]);
                    }
                }
            }
            // side faces, per (face, edge point): face point e + PL k lifts
            // onto layer k
#pragma unroll 1
            for (int u = 0; u < 3 * PL; ++u) {
#pragma unroll
                for (int k = 0; k < PL; ++k) {
                    const int t = 2 * NT + u / PL * (PL * PL) + u % PL + PL * k;
                    const Real jump = jump_at(t);
#pragma unroll
                    for (int m = 0; m < NT; ++m) {
                        const int i = m + NT * k;
                        r[i] = fma(-op.lift[t * NS + i], jump, r[i]);
                    }
                }
            }
        } else {
#pragma unroll 1
            for (int t = 0; t < NFT; ++t) {
                const Real jump = jump_at(t);
#pragma unroll
                for (int i = 0; i < NS; ++i) r[i] = fma(-op.lift[t * NS + i], jump, r[i]);
            }
        }
    } else {
#pragma unroll 4
        for (int i = 0; i < NS; ++i) sf[i][lane] = ldo(fE + i * nu, ko);
#pragma unroll 1
        for (int i = 0; i < NS; ++i) {
            Real acc = Real(0);
#pragma unroll 4
            for (int j = 0; j < NS; ++j) {
                const Real w = c[0] * op.D[i * NS + j] + c[1] * op.D[(NS + i) * NS + j] + c[2] * op.D[(2 * NS + i) * NS + j];
                acc = fma(w, sf[j][lane], acc);
            }
            sa[i][lane] = -acc;
        }
#pragma unroll 1
        for (int t = 0; t < NFT; ++t) {
            const Real jump = jump_at(t);
#pragma unroll 4
            for (int i = 0; i < NS; ++i) sa[i][lane] -= op.lift[t * NS + i] * jump;
        }
    }
    auto res = [&](int i) -> Real {
        if constexpr (REG) return r[i];
        else return sa[i][lane];
    };
    auto val = [&](int i) -> Real {
        if constexpr (REG) return fv[i];
        else return sf[i][lane];
    };
    if (MODE == GMODE_RESID) {
        Real *R = reinterpret_cast<Real *>(A.sa.fout) + p0 * nu;
        if (act)
#pragma unroll
            for (int i = 0; i < NS; ++i) sto(R + i * nu, ko, res(i));
        return;
    }
    // collision source and the Runge-Kutta combination, point by point
    const Real dt = (Real)A.sa.dt;
    const bool collide = A.sa.collide;
    const bool useX = A.sa.scheme == 0 ? A.sa.alpha != 0.0 : A.sa.lsA != 0.0;
    const Real *XE = reinterpret_cast<const Real *>(A.sa.scheme == 0 ? A.sa.fn : A.sa.dF) + p0 * nu;
    Real *outE = reinterpret_cast<Real *>(A.sa.fout) + p0 * nu;
    Real *dFE = reinterpret_cast<Real *>(A.sa.dF) + p0 * nu;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        const Real fq = val(i);
        Real L = res(i);
        if (collide) {
            const cptr<double> q = (cptr<double>)A.sa.eq + (p0 + i) * kEqW;
            const double c0 = ud[0] - q[EQ_V], c1 = ud[1] - q[EQ_V + 1], c2 = ud[2] - q[EQ_V + 2];
            double t0_ = -0.5 * q[EQ_B] * c0;
            t0_ = fma(-q[EQ_B + 3], c1, t0_);
            t0_ = fma(-q[EQ_B + 4], c2, t0_);
            double t1 = -0.5 * q[EQ_B + 1] * c1;
            t1 = fma(-q[EQ_B + 5], c2, t1);
            const double t2 = -0.5 * q[EQ_B + 2] * c2;
            double E = fma(c0, t0_, q[EQ_C0]);
            E = fma(c1, t1, E);
            E = fma(c2, t2, E);
            L += (gexp<Real>(E) - fq) * (Real)q[EQ_INVTAU];
        }
        const Real xv = useX ? ldo(XE + i * nu, ko) : Real(0);
        double fod;
        if (A.sa.scheme == 0) {
            fod = A.sa.beta * ((double)fq + (double)(dt * L));
            if (useX) fod = fma(A.sa.alpha, (double)xv, fod);
        } else {
            Real dd = dt * L;
            if (useX) dd += (Real)A.sa.lsA * xv;
            if (act && A.sa.keep_dF) sto(dFE + i * nu, ko, dd);
            fod = fma(A.sa.lsB, (double)dd, (double)fq);
        }
        Real fo;
        if constexpr (sizeof(Real) == 4)
            fo = round_stochastic(fod, round_bits(A.sa.seed, (uint32_t)(p0 + i), (uint32_t)k));
        else
            fo = (Real)fod;
        sf[i][lane] = fo;
        if (act) sto(outE + i * nu, ko, fo);
    }
    if (A.do_traces && act) {
        Real *trO = reinterpret_cast<Real *>(A.sa.tr_out) + t0 * nu;
#pragma unroll 1
        for (int t = 0; t < NFT; ++t) sto(trO + t * nu, ko, sf[fnode[t]][lane]);
    }
}

// Traces of f: its values at the face points.
template <typename Real, int NS, int NFT>
__global__ __launch_bounds__(kGWave) void k_mix_traces(const MixArgs A, const Real *__restrict__ f, Real *__restrict__ tr) {
    const int64_t e = A.elems[blockIdx.x / A.nvw];
    const int k = (int)(blockIdx.x % A.nvw) * kGWave + threadIdx.x;
    if (k >= A.nu) return;
    const int64_t nu = A.nu, p0 = A.poff[e], t0 = A.toff[e];
#pragma unroll 1
    for (int t = 0; t < NFT; ++t) tr[(t0 + t) * nu + k] = f[(p0 + A.fnode[t]) * nu + k];
}

template <typename Real, int NS, int NFT, int PL = 0>
int mix_launch(fr_dvm *h, int mode, const MixArgs &A, unsigned blocks) {
    if (mode == 0)
        hipLaunchKernelGGL((k_mix_traces<Real, NS, NFT>), dim3(blocks), dim3(kGWave), 0, h->stream, A,
                           reinterpret_cast<const Real *>(A.sa.f), reinterpret_cast<Real *>(A.sa.tr_out));
    else if (mode == GMODE_RESID)
        hipLaunchKernelGGL((k_mix_stage<Real, NS, NFT, GMODE_RESID, PL>), dim3(blocks), dim3(kGWave), 0, h->stream, A);
    else
        hipLaunchKernelGGL((k_mix_stage<Real, NS, NFT, GMODE_STAGE, PL>), dim3(blocks), dim3(kGWave), 0, h->stream, A);
    return gcheck(h, "mixed-mesh kernel");
}

// (type, order) -> the kernel instantiation for its point counts
template <typename Real>
int mix_dispatch(fr_dvm *h, int mode, const MixArgs &A, int t, const MixType &T, unsigned blocks) {
    const int key = 10 * t + h->p;
    int ns = 0, nft = 0, rc = FR_DVM_EUNSUPPORTED;
    switch (key) {
        case 1: ns = 8; nft = 24; rc = mix_launch<Real, 8, 24>(h, mode, A, blocks); break;
        case 2: ns = 27; nft = 54; rc = mix_launch<Real, 27, 54>(h, mode, A, blocks); break;
        case 3: ns = 64; nft = 96; rc = mix_launch<Real, 64, 96>(h, mode, A, blocks); break;
        case 11: ns = 6; nft = 18; rc = mix_launch<Real, 6, 18, 2>(h, mode, A, blocks); break;
        case 12: ns = 18; nft = 39; rc = mix_launch<Real, 18, 39, 3>(h, mode, A, blocks); break;
        case 13: ns = 40; nft = 68; rc = mix_launch<Real, 40, 68, 4>(h, mode, A, blocks); break;
        case 21: ns = 4; nft = 12; rc = mix_launch<Real, 4, 12>(h, mode, A, blocks); break;
        case 22: ns = 10; nft = 24; rc = mix_launch<Real, 10, 24>(h, mode, A, blocks); break;
        case 23: ns = 20; nft = 40; rc = mix_launch<Real, 20, 40>(h, mode, A, blocks); break;
        default: return h->fail(FR_DVM_EUNSUPPORTED, "mixed-mesh element type / order");
    }
    (void)ns;
    (void)nft;
    return rc;
}

template <typename Real>
int mix_run(fr_dvm *h, int mode, const StageArgs &sa, int do_traces, int do_moments) {
    const Mixed &mx = *h->mx;
    MixArgs A;
    std::memset(&A, 0, sizeof(A));
    A.vg = h->vg;
    A.nu = h->vg.nu;
    A.nvw = (A.nu + kGWave - 1) / kGWave;
    A.poff = mx.d_poff;
    A.toff = mx.d_toff;
    A.tnb = mx.d_tnb;
    A.geo = mx.d_geo;
    A.geof = mx.d_geof;
    A.sa = sa;
    A.do_traces = do_traces;
    int rc;
    if (mode != 0 || do_traces) {
        for (int t = 0; t < 3; ++t) {
            const MixType &T = mx.t[t];
            if (T.elems.empty()) continue;
            const int key_ns[3][4] = {{0, 8, 27, 64}, {0, 6, 18, 40}, {0, 4, 10, 20}};
            if (T.ns != key_ns[t][h->p]) return h->fail(FR_DVM_EINVAL, "mixed-mesh operator size");
            A.elems = T.d_elems;
            A.D = T.d_D;
            A.lift = T.d_lift;
            A.Df = T.d_Df;
            A.liftf = T.d_liftf;
            A.fnode = T.d_fnode;
            A.ffac = T.d_ffac;
            if ((rc = mix_dispatch<Real>(h, mode, A, t, T, (unsigned)(T.elems.size() * A.nvw)))) return rc;
        }
    }
    const bool moments = (mode == 0 || mode == GMODE_STAGE) && do_moments;
    if (!moments) return FR_DVM_OK;
    // moments of every point: the general-mesh reduction over the velocity axis
    GenArgs G;
    std::memset(&G, 0, sizeof(G));
    G.vg = h->vg;
    G.nu = h->vg.nu;
    G.ncomp = 1;
    G.nut = G.nu;
    G.wax = h->d_wax;
    const Real *src = reinterpret_cast<const Real *>(mode == 0 ? sa.f : sa.fout);
    const unsigned npts = (unsigned)mx.npts;
    if (h->nmom == 5)
        hipLaunchKernelGGL((k_gen_moments<Real, 5>), dim3(gen_moment_grid(npts)), dim3(64 * kMomPts), 0, h->stream, G, src, sa.Q, (int64_t)npts);
    else if (h->nmom == 10)
        hipLaunchKernelGGL((k_gen_moments<Real, 10>), dim3(gen_moment_grid(npts)), dim3(64 * kMomPts), 0, h->stream, G, src, sa.Q, (int64_t)npts);
    else
        return h->fail(FR_DVM_EUNSUPPORTED, "mixed meshes need a monatomic gas");
    return gcheck(h, "moment kernel");
}

}  // namespace

int launch_fr_mixed(fr_dvm *h, int mode, const StageArgs &sa, int do_traces, int do_moments) {
    if (sa.e0 != 0 || sa.ecount != 0) return h->fail(FR_DVM_EINVAL, "element ranges need an axis-aligned box mesh");
    return h->prm.precision == FR_DVM_FP64 ? mix_run<double>(h, mode, sa, do_traces, do_moments)
                                           : mix_run<float>(h, mode, sa, do_traces, do_moments);
}

int launch_fr_gen(fr_dvm *h, int mode, const StageArgs &sa, int do_traces, int do_moments) {
    if (sa.e0 != 0 || sa.ecount != 0) return h->fail(FR_DVM_EINVAL, "element ranges need an axis-aligned box mesh");
    GenArgs A;
    std::memset(&A, 0, sizeof(A));
    for (int i = 0; i < kMaxN * kMaxN; ++i) {
        A.od.D[i] = h->ops.D[i];
        A.of.D[i] = (float)h->ops.D[i];
    }
    for (int s = 0; s < 2; ++s)
        for (int m = 0; m < kMaxN; ++m) {
            A.od.lam[s][m] = h->ops.lam[s][m];
            A.of.lam[s][m] = (float)h->ops.lam[s][m];
            A.od.corr[s][m] = h->ops.corr[s][m];
            A.of.corr[s][m] = (float)h->ops.corr[s][m];
        }
    A.vg = h->vg;
    A.nu = h->vg.nu;
    A.ncomp = h->ncomp;
    A.nut = A.nu * A.ncomp;
    A.nvb = (A.nut + kGBlock - 1) / kGBlock;
    A.nvw = (A.nut + kGWave - 1) / kGWave;
    A.gwall = 0.5 * h->delta * h->prm.theta_wall;
    A.gfp = h->d_gfp;
    A.wax = h->d_wax;
    A.wJ = h->d_wq3J;
    A.S = h->d_S;
    A.ijac = h->d_ijac;
    A.nf = h->d_nf;
    A.Sf = h->d_Sf;
    A.ijacf = h->d_ijacf;
    A.nff = h->d_nff;
    A.conn = h->d_conn;
    A.wall = h->d_wall;
    A.rw = h->d_rw;
    A.mw = h->d_mw;
    A.finf = h->d_finf;
    A.sa = sa;
    A.do_traces = do_traces;
    return h->prm.precision == FR_DVM_FP64 ? gen_p<double>(h, mode, A, do_moments)
                                           : gen_p<float>(h, mode, A, do_moments);
}

}  // namespace frdvm
