// Conservative discrete equilibrium (FP64 Newton), stand-alone collision,
// moment output and global totals (gfx950).
//
// Paper, Section "Numerical method", eq. (discrete_compatibility): the
// modified equilibrium g' must have exactly the discrete moments of f,
// M.(g' psi) = M.(f psi).  Following Mieussens it is the analytic
// equilibrium at a modified state Q', i.e. an exponential of a quadratic in
// u, found per solution point by a small nonlinear solve (Newton).  Section
// "Governing equations": tau = mu/(Pr P), ES-BGK tensor
// T = theta/Pr I + (1 - 1/Pr) Pi/rho.
//
// Formulation (the same reading as the CPU oracle): in the frame
// c = (u - U)/sqrt(theta) with weights wt = w theta^-3/2 the five equations
// are sum_k wt_k (1, c_k, |c_k|^2/2) exp(z0 + z.c_k - z4 q(c_k)/2) =
// (1, 0, 0, 0, 3/2), q = |c|^2 (BGK) or c^T A c with A = theta T^-1 (ES-BGK),
// and g' = rho wt exp(...).
//
// BGK kernel: one thread per point.  On a tensor velocity grid the BGK
// exponential factorises per axis, so each Newton iteration costs 3 n_v
// exponentials and 1-D power sums instead of n_v^3 terms.
// ES kernel: 32 lanes per point (two points per wave), lanes over velocity
// nodes or node pairs, butterfly reduction of the 18 sums (lane-symmetric:
// every lane gets the same bits); the iteration state lives in LDS.
// Starting points: cold (continuous equilibrium of the moments), warm (the
// previous solution at the point) or learned (cold + a correction predicted
// by the MLP kernels; the start with the smaller residual is kept, so the
// learned start never costs more than one extra evaluation).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "frdvm_common.h"
#include "frdvm_dev.h"

namespace frdvm {

namespace {

struct NewtonArgs {
    VGrid vg;
    int64_t npts;
    int nmom;
    const double *wax;   // [3][64]
    const double *Q;     // [npts][nmom]
    double *eq;          // [npts][kEqW]
    double *z;           // [npts][5]
    double *prim;        // [npts][5]
    unsigned long long *stats;  // [kHist] histogram, [kHist] fallback, [kHist+1] ES guard
    unsigned long long *maxres;
    int32_t *pt_iters;   // optional per-point outputs
    int32_t *pt_evals;
    int32_t *pt_status;
    double *pt_resid;
    double Pr, mu_ref, theta_ref, omega, theta_s;
    int visc_law;
    double tol;
    int max_iter;
    int guess;
    const float *dz_guess;  // [npts][5] learned correction (guess == MLP)
    int use_fact;           // ES: factorised sums with per-point LDS tables
    double delta;           // internal degrees of freedom (the reduced pair)
    double *gfp;            // [npts] delta theta / 2 per point (pair only, else null)
};

// Total energy of a moment record: E (BGK), half the trace of the raw second
// moments (ES), plus the integral of G in the last slot for the reduced pair
// (records of 6 / 11 values).
__device__ __forceinline__ double record_energy(const double *q, int nmom) {
    switch (nmom) {
        case 5: return q[4];
        case 6: return q[4] + q[5];
        case 10: return 0.5 * (q[4] + q[5] + q[6]);
        default: return 0.5 * (q[4] + q[5] + q[6]) + q[10];
    }
}

constexpr double kTwoPi = 6.283185307179586476925286766559;
// Line search: the step is halved after each rejected trial point (z4 <= 0 or
// too little decrease of |r|_2); a solve may reject at most this many trial
// points in total, then it stops (fallback unless at the rounding floor).
constexpr int kRejectBudget = 40;

// Velocity node umin + i du, rounded as two separate operations (no FMA
// contraction) so that every kernel sees the node values the host sees.
__device__ __forceinline__ double gridu(const VGrid &vg, int d, int i) {
    return __dadd_rn(vg.umin[d], __dmul_rn((double)i, vg.du[d]));
}

__device__ double viscosity(const NewtonArgs &A, double th) {
    if (A.visc_law == 1)
        return A.mu_ref * pow(th / A.theta_ref, 1.5) * (A.theta_ref + A.theta_s) / (th + A.theta_s);
    return A.mu_ref * pow(th / A.theta_ref, A.omega);
}

// Gaussian elimination with partial pivoting on a 5x5 system.  Every loop is
// unrolled so the row exchange is a set of selects on registers.
__device__ __forceinline__ bool solve5(const double J[5][5], const double b[5], double x[5]) {
    double M[5][6];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
#pragma unroll
        for (int j = 0; j < 5; ++j) M[i][j] = J[i][j];
        M[i][5] = b[i];
    }
    bool ok = true;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        double best = fabs(M[c][c]);
        int piv = c;
#pragma unroll
        for (int r = c + 1; r < 5; ++r)
            if (fabs(M[r][c]) > best) { best = fabs(M[r][c]); piv = r; }
        ok = ok && (best > 0.0);
#pragma unroll
        for (int r = c + 1; r < 5; ++r) {
            const bool sw = (r == piv);
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                double a = M[c][j], bb = M[r][j];
                M[c][j] = sw ? bb : a;
                M[r][j] = sw ? a : bb;
            }
        }
        const double inv = 1.0 / M[c][c];
#pragma unroll
        for (int r = c + 1; r < 5; ++r) {
            const double fct = M[r][c] * inv;
#pragma unroll
            for (int j = c; j < 6; ++j) M[r][j] -= fct * M[c][j];
        }
    }
#pragma unroll
    for (int i = 4; i >= 0; --i) {
        double s = M[i][5];
#pragma unroll
        for (int j = i + 1; j < 5; ++j) s -= M[i][j] * x[j];
        x[i] = s / M[i][i];
    }
    return ok;
}

__device__ __forceinline__ double norm2_5(const double r[5]) {
    return sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3] + r[4] * r[4]);
}
__device__ __forceinline__ double normi_5(const double r[5]) {
    double m = 0;
#pragma unroll
    for (int a = 0; a < 5; ++a) m = fmax(m, fabs(r[a]));
    return m;
}

// Raw sums over the velocity grid:
//   S0 = sum wt e, Sc_i = sum wt c_i e, Scc (xx yy zz xy xz yz), Sq = sum wt q e,
//   Scq_i = sum wt c_i q e, Sc2c_i = sum wt |c|^2 c_i e, Sc2q = sum wt |c|^2 q e.
struct Sums {
    double S0, Sc[3], Scc[6], Sq, Scq[3], Sc2c[3], Sc2q;
};

// Residual and Jacobian; rows psi = (1, c, |c|^2/2), columns d/dz = (1, c, -q/2).
__device__ __forceinline__ void assemble(const Sums &s, double r[5], double J[5][5]) {
    const double c2 = s.Scc[0] + s.Scc[1] + s.Scc[2];
    r[0] = s.S0 - 1.0;
    r[1] = s.Sc[0];
    r[2] = s.Sc[1];
    r[3] = s.Sc[2];
    r[4] = 0.5 * c2 - 1.5;
    J[0][0] = s.S0; J[0][1] = s.Sc[0]; J[0][2] = s.Sc[1]; J[0][3] = s.Sc[2]; J[0][4] = -0.5 * s.Sq;
    J[1][0] = s.Sc[0]; J[1][1] = s.Scc[0]; J[1][2] = s.Scc[3]; J[1][3] = s.Scc[4]; J[1][4] = -0.5 * s.Scq[0];
    J[2][0] = s.Sc[1]; J[2][1] = s.Scc[3]; J[2][2] = s.Scc[1]; J[2][3] = s.Scc[5]; J[2][4] = -0.5 * s.Scq[1];
    J[3][0] = s.Sc[2]; J[3][1] = s.Scc[4]; J[3][2] = s.Scc[5]; J[3][3] = s.Scc[2]; J[3][4] = -0.5 * s.Scq[2];
    J[4][0] = 0.5 * c2; J[4][1] = 0.5 * s.Sc2c[0]; J[4][2] = 0.5 * s.Sc2c[1]; J[4][3] = 0.5 * s.Sc2c[2];
    J[4][4] = -0.25 * s.Sc2q;
}

// BGK sums by axis factorisation: e = exp(z0) prod_d exp(z_d c_d - z4 c_d^2 / 2).
__device__ void sums_bgk(const NewtonArgs &A, const double U[3], double ist, const double z[5], Sums &s) {
    double m[3][5];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0;
        const int nv = A.vg.nv[d];
        const double zd = z[1 + d], hz = 0.5 * z[4];
        for (int i = 0; i < nv; ++i) {
            const double c = (gridu(A.vg, d, i) - U[d]) * ist;
            const double ev = A.wax[64 * d + i] * ist * exp(c * (zd - hz * c));
            double t = ev;
            a0 += t; t *= c;
            a1 += t; t *= c;
            a2 += t; t *= c;
            a3 += t; t *= c;
            a4 += t;
        }
        m[d][0] = a0; m[d][1] = a1; m[d][2] = a2; m[d][3] = a3; m[d][4] = a4;
    }
    const double K = exp(z[0]) * m[0][0] * m[1][0] * m[2][0];
    double Pn[3][5];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double inv = 1.0 / m[d][0];
#pragma unroll
        for (int a = 0; a < 5; ++a) Pn[d][a] = m[d][a] * inv;
    }
    s.S0 = K;
#pragma unroll
    for (int i = 0; i < 3; ++i) s.Sc[i] = K * Pn[i][1];
    s.Scc[0] = K * Pn[0][2]; s.Scc[1] = K * Pn[1][2]; s.Scc[2] = K * Pn[2][2];
    s.Scc[3] = K * Pn[0][1] * Pn[1][1];
    s.Scc[4] = K * Pn[0][1] * Pn[2][1];
    s.Scc[5] = K * Pn[1][1] * Pn[2][1];
    s.Sq = s.Scc[0] + s.Scc[1] + s.Scc[2];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double t = 0;
#pragma unroll
        for (int mm = 0; mm < 3; ++mm) t += (mm == i) ? Pn[i][3] : Pn[i][1] * Pn[mm][2];
        s.Scq[i] = K * t;
        s.Sc2c[i] = K * t;
    }
    double t4 = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) t4 += (a == b) ? Pn[a][4] : Pn[a][2] * Pn[b][2];
    s.Sc2q = K * t4;
}

// ES sums: kLpp lanes per solution point (two points per wave), reduced by
// a butterfly inside each half-wave.
constexpr int kLpp = 32;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = kLpp / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, kLpp);
    return v;
}

// ES sums over all velocity nodes: lane-strided, butterfly reduced.  With
// jac == false only the residual sums S0, Sc and the trace of Scc (stored in
// Scc[0]) are formed.
__device__ void sums_es(const NewtonArgs &A, int lane, const double U[3], double ist, double wscale,
                        const double Am[3][3], const double z[5], Sums &s, bool jac) {
    double acc[18];
#pragma unroll
    for (int a = 0; a < 18; ++a) acc[a] = 0.0;
    const VGrid &vg = A.vg;
    for (int k = lane; k < vg.nu; k += kLpp) {
        const int i = k % vg.nv[0], j = (k / vg.nv[0]) % vg.nv[1], l = k / (vg.nv[0] * vg.nv[1]);
        const double c0 = (gridu(vg, 0, i) - U[0]) * ist;
        const double c1 = (gridu(vg, 1, j) - U[1]) * ist;
        const double c2 = (gridu(vg, 2, l) - U[2]) * ist;
        const double q = Am[0][0] * c0 * c0 + Am[1][1] * c1 * c1 + Am[2][2] * c2 * c2 +
                         2.0 * (Am[0][1] * c0 * c1 + Am[0][2] * c0 * c2 + Am[1][2] * c1 * c2);
        const double w = A.wax[i] * A.wax[64 + j] * A.wax[128 + l] * wscale;
        const double ev = w * exp(z[0] + z[1] * c0 + z[2] * c1 + z[3] * c2 - 0.5 * z[4] * q);
        const double cc = c0 * c0 + c1 * c1 + c2 * c2;
        acc[0] += ev;
        acc[1] += ev * c0; acc[2] += ev * c1; acc[3] += ev * c2;
        if (!jac) {
            acc[4] += ev * cc;
            continue;
        }
        const double eq_ = ev * q, ec = ev * cc;
        acc[4] += ev * c0 * c0; acc[5] += ev * c1 * c1; acc[6] += ev * c2 * c2;
        acc[7] += ev * c0 * c1; acc[8] += ev * c0 * c2; acc[9] += ev * c1 * c2;
        acc[10] += eq_;
        acc[11] += eq_ * c0; acc[12] += eq_ * c1; acc[13] += eq_ * c2;
        acc[14] += ec * c0; acc[15] += ec * c1; acc[16] += ec * c2;
        acc[17] += ec * q;
    }
    s.S0 = wave_sum(acc[0]);
#pragma unroll
    for (int d = 0; d < 3; ++d) s.Sc[d] = wave_sum(acc[1 + d]);
    if (!jac) {
        s.Scc[0] = wave_sum(acc[4]);
        s.Scc[1] = s.Scc[2] = 0.0;
        return;
    }
#pragma unroll
    for (int a = 0; a < 6; ++a) s.Scc[a] = wave_sum(acc[4 + a]);
    s.Sq = wave_sum(acc[10]);
#pragma unroll
    for (int d = 0; d < 3; ++d) s.Scq[d] = wave_sum(acc[11 + d]);
#pragma unroll
    for (int d = 0; d < 3; ++d) s.Sc2c[d] = wave_sum(acc[14 + d]);
    s.Sc2q = wave_sum(acc[17]);
}

// ---- factorised ES sums -------------------------------------------------
// On a tensor grid the exponent z0 + z.c - z4 c^T A c / 2 splits into the
// one-axis factors X(i), Y(j), Z(l) and the cross factors exp(k01 c0 c1),
// exp(k02 c0 c2), exp(k12 c1 c2) (k_ab = -z4 A_ab).  The first cross factor
// is tabulated, P(i,j).  The product of the other two,
// G(i,j,l) = exp((k02 c0_i + k12 c1_j) c2_l), is geometric in l on a uniform
// grid with start G0(i) H0(j) and ratio Ra(i) Rb(j), so it is generated along
// l and needs no table: 3n + 3n + n + 2n exponentials per evaluation.  The
// sums follow from T_e(i,j) = sum_l Z c2^e G and the pair sums, reduced over
// the lanes of the point.

// Layout of one point's table region (doubles); rows of P are padded to an
// odd length to spread LDS banks.
struct FactLayout {
    int n0, n1, n2, ld1;  // ld1 = row length of P (over j)
    int c0, c1, c2, X, Y, Zc, P, G0, Ra, H0, Rb, total;
};

__host__ __device__ inline FactLayout fact_layout(const VGrid &vg) {
    FactLayout L;
    L.n0 = vg.nv[0];
    L.n1 = vg.nv[1];
    L.n2 = vg.nv[2];
    L.ld1 = L.n1 | 1;
    int o = 0;
    L.c0 = o; o += L.n0;
    L.c1 = o; o += L.n1;
    L.c2 = o; o += L.n2;
    L.X = o; o += L.n0;
    L.Y = o; o += L.n1;
    L.Zc = o; o += 5 * L.n2;
    L.P = o; o += L.n0 * L.ld1;
    L.G0 = o; o += L.n0;
    L.Ra = o; o += L.n0;
    L.H0 = o; o += L.n1;
    L.Rb = o; o += L.n1;
    L.total = o;
    return L;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = kLpp / 2; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, kLpp));
    return v;
}

__device__ __forceinline__ void lds_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Quadratic-form entries a pair finish needs: A00, A11, A22, 2A01, 2A02, 2A12.
struct QuadA {
    double a00, a11, a22, t01, t02, t12;
};

// B pairs p0 + kLpp b (all < n0 n1) of one lane: T_e = sum_l Z c2^e G for
// e < NE (5 for the full sums, 3 for the residual sums), then the pairs'
// contributions to the 18 (5) sums.  Returns the largest |exponent| of G
// over the pairs (G is exact at both ends of l, hence everywhere between).
template <int B, int NE>
__device__ __forceinline__ double pair_block(const FactLayout &L, const double *tb, int p0, double k02, double k12,
                                             const QuadA &q, double acc[18]) {
    constexpr bool JAC = NE == 5;
    double g[B], gr[B], T[B][NE];
    int ii[B], jj[B];
    double gmax = 0.0;
    const double c2a = tb[L.c2], c2b = tb[L.c2 + L.n2 - 1];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const unsigned p = (unsigned)(p0 + kLpp * b);  // non-negative: unsigned division is shorter
        ii[b] = (int)(p % (unsigned)L.n0);
        jj[b] = (int)(p / (unsigned)L.n0);
        const double kap = k02 * tb[L.c0 + ii[b]] + k12 * tb[L.c1 + jj[b]];
        gmax = fmax(gmax, fmax(fabs(kap * c2a), fabs(kap * c2b)));
        g[b] = tb[L.G0 + ii[b]] * tb[L.H0 + jj[b]];
        gr[b] = tb[L.Ra + ii[b]] * tb[L.Rb + jj[b]];
#pragma unroll
        for (int e = 0; e < NE; ++e) T[b][e] = 0.0;
    }
    for (int l = 0; l < L.n2; ++l) {
        const double *zc = tb + L.Zc + 5 * l;
        double zl[NE];
#pragma unroll
        for (int e = 0; e < NE; ++e) zl[e] = zc[e];
#pragma unroll
        for (int b = 0; b < B; ++b) {
#pragma unroll
            for (int e = 0; e < NE; ++e) T[b][e] = fma(zl[e], g[b], T[b][e]);
            g[b] *= gr[b];
        }
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int i = ii[b], j = jj[b];
        const double T0 = T[b][0], T1 = T[b][1], T2 = T[b][2];
        const double c0 = tb[L.c0 + i], c1 = tb[L.c1 + j];
        const double bb = tb[L.X + i] * tb[L.Y + j] * tb[L.P + i * L.ld1 + j];
        const double r2 = c0 * c0 + c1 * c1;
        acc[0] += bb * T0;
        acc[1] += bb * c0 * T0; acc[2] += bb * c1 * T0; acc[3] += bb * T1;
        if constexpr (!JAC) {
            acc[4] += bb * (r2 * T0 + T2);
        } else {
            const double T3 = T[b][NE > 3 ? 3 : 0], T4 = T[b][NE > 4 ? 4 : 0];
            const double qa = c0 * (q.a00 * c0 + q.t01 * c1) + q.a11 * c1 * c1, qb = q.t02 * c0 + q.t12 * c1;
            const double q0 = qa * T0 + qb * T1 + q.a22 * T2;    // sum q
            const double q1 = qa * T1 + qb * T2 + q.a22 * T3;    // sum c2 q
            const double q2 = qa * T2 + qb * T3 + q.a22 * T4;    // sum c2^2 q
            const double s2 = r2 * T0 + T2;                      // sum |c|^2
            acc[4] += bb * c0 * c0 * T0; acc[5] += bb * c1 * c1 * T0; acc[6] += bb * T2;
            acc[7] += bb * c0 * c1 * T0; acc[8] += bb * c0 * T1; acc[9] += bb * c1 * T1;
            acc[10] += bb * q0;
            acc[11] += bb * c0 * q0; acc[12] += bb * c1 * q0; acc[13] += bb * q1;
            acc[14] += bb * c0 * s2; acc[15] += bb * c1 * s2; acc[16] += bb * (r2 * T1 + T3);
            acc[17] += bb * (r2 * q0 + q2);
        }
    }
    return gmax;
}

// All n0 n1 pairs of the point: full passes of four pairs per lane, then the
// remainder one pair per lane.
template <int NE>
__device__ __forceinline__ double pair_sums(const FactLayout &L, const double *tb, int lane, double k02, double k12,
                                            const QuadA &q, double acc[18]) {
    const int nP = L.n0 * L.n1;
    const int full = nP / (2 * kLpp) * (2 * kLpp);
    double gmax = 0.0;
    for (int p0 = lane; p0 < full; p0 += 2 * kLpp) gmax = fmax(gmax, pair_block<2, NE>(L, tb, p0, k02, k12, q, acc));
    for (int p0 = full + lane; p0 < nP; p0 += kLpp) gmax = fmax(gmax, pair_block<1, NE>(L, tb, p0, k02, k12, q, acc));
    return gmax;
}

// Returns false (and leaves s untouched) when a factor exponent exceeds the
// safe range; the caller then uses the direct sum.  jac as for sums_es.
__device__ bool sums_es_fact(const NewtonArgs &A, int lane, double *tb, const double U[3], double ist,
                             const double Am[3][3], const double z[5], Sums &s, bool jac) {
    // per-evaluation values: nothing derived from the lane or the frame is
    // hoisted out of the caller's Newton loop (it would stay live across it)
    asm volatile("" : "+v"(lane), "+v"(ist));
    const VGrid &vg = A.vg;
    const FactLayout L = fact_layout(vg);
    const double hz = 0.5 * z[4];
    const double k01 = -z[4] * Am[0][1], k02 = -z[4] * Am[0][2], k12 = -z[4] * Am[1][2];
    // c2 at the first node and the c2 spacing (the G recurrence runs along l)
    const double c2a = (gridu(vg, 2, 0) - U[2]) * ist, dl2 = vg.du[2] * ist;
    // largest exponent of a direct factor (X, Y, Z, P: an underflow there is
    // a true underflow) and largest |exponent| of a G factor (its start and
    // ratio tables must neither overflow nor underflow)
    double amax = -1e300;
    lds_wave_sync();  // previous evaluation's readers are done with the tables
    // one-axis tables, axis by axis (an axis index varying across lanes would
    // put the small per-point arrays U, z, Am into scratch memory)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int nd = d == 0 ? L.n0 : (d == 1 ? L.n1 : L.n2);
        const int oc = d == 0 ? L.c0 : (d == 1 ? L.c1 : L.c2);
        for (int i = lane; i < nd; i += kLpp) {
            const double c = (gridu(vg, d, i) - U[d]) * ist;
            double arg = c * (z[1 + d] - hz * Am[d][d] * c);
            if (d == 0) arg += z[0];
            amax = fmax(amax, arg);
            const double v = A.wax[64 * d + i] * ist * exp(arg);
            tb[oc + i] = c;
            if (d == 0) {
                tb[L.X + i] = v;
                const double g0 = k02 * c * c2a, gr = k02 * c * dl2;
                amax = fmax(amax, fmax(fabs(g0), fabs(gr)));
                tb[L.G0 + i] = exp(g0);
                tb[L.Ra + i] = exp(gr);
            } else if (d == 1) {
                tb[L.Y + i] = v;
                const double h0 = k12 * c * c2a, hr = k12 * c * dl2;
                amax = fmax(amax, fmax(fabs(h0), fabs(hr)));
                tb[L.H0 + i] = exp(h0);
                tb[L.Rb + i] = exp(hr);
            } else {
                double p = v;
#pragma unroll
                for (int e = 0; e < 5; ++e) { tb[L.Zc + 5 * i + e] = p; p *= c; }
            }
        }
    }
    lds_wave_sync();
    // P(i,j) = exp(k01 c0_i c1_j): along a row the exponent is affine in j,
    // so one lane fills a row by a geometric recurrence from its larger end
    // (2 exponentials per row; values only shrink along the recurrence, so an
    // underflow is a true underflow).
    for (int i = lane; i < L.n0; i += kLpp) {
        const double kc = k01 * tb[L.c0 + i];
        const int nb = L.n1;
        double *dst = tb + L.P + i * L.ld1;
        const double a0 = kc * tb[L.c1], a1 = kc * tb[L.c1 + nb - 1];
        amax = fmax(amax, fmax(a0, a1));
        const double step = nb > 1 ? fabs(a1 - a0) / (nb - 1) : 0.0;
        const double ratio = exp(-step);
        const bool up = a1 > a0;  // the larger end is the last node
        double v = exp(up ? a1 : a0);
        for (int m = 0; m < nb; ++m) {
            dst[up ? nb - 1 - m : m] = v;
            v *= ratio;
        }
    }
    lds_wave_sync();
    const QuadA q = {Am[0][0], Am[1][1], Am[2][2], 2.0 * Am[0][1], 2.0 * Am[0][2], 2.0 * Am[1][2]};
    double acc[18];
#pragma unroll
    for (int a = 0; a < 18; ++a) acc[a] = 0.0;
    const double gmax = jac ? pair_sums<5>(L, tb, lane, k02, k12, q, acc) : pair_sums<3>(L, tb, lane, k02, k12, q, acc);
    if (wave_max(fmax(amax, gmax)) > 600.0) return false;
    s.S0 = wave_sum(acc[0]);
#pragma unroll
    for (int d = 0; d < 3; ++d) s.Sc[d] = wave_sum(acc[1 + d]);
    if (!jac) {
        s.Scc[0] = wave_sum(acc[4]);
        s.Scc[1] = s.Scc[2] = 0.0;
        return true;
    }
#pragma unroll
    for (int a = 0; a < 6; ++a) s.Scc[a] = wave_sum(acc[4 + a]);
    s.Sq = wave_sum(acc[10]);
#pragma unroll
    for (int d = 0; d < 3; ++d) s.Scq[d] = wave_sum(acc[11 + d]);
#pragma unroll
    for (int d = 0; d < 3; ++d) s.Sc2c[d] = wave_sum(acc[14 + d]);
    s.Sc2q = wave_sum(acc[17]);
    return true;
}

// Smallest eigenvalue of a symmetric 3x3 matrix (closed form, trigonometric).
__device__ double sym3_min_eig(const double T[3][3]) {
    const double p1 = T[0][1] * T[0][1] + T[0][2] * T[0][2] + T[1][2] * T[1][2];
    const double q = (T[0][0] + T[1][1] + T[2][2]) / 3.0;
    if (p1 == 0.0) return fmin(T[0][0], fmin(T[1][1], T[2][2]));
    const double p2 = (T[0][0] - q) * (T[0][0] - q) + (T[1][1] - q) * (T[1][1] - q) +
                      (T[2][2] - q) * (T[2][2] - q) + 2.0 * p1;
    const double p = sqrt(p2 / 6.0);
    double B[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) B[i][j] = (T[i][j] - (i == j ? q : 0.0)) / p;
    const double detB = B[0][0] * (B[1][1] * B[2][2] - B[1][2] * B[2][1]) -
                        B[0][1] * (B[1][0] * B[2][2] - B[1][2] * B[2][0]) +
                        B[0][2] * (B[1][0] * B[2][1] - B[1][1] * B[2][0]);
    const double r = fmin(1.0, fmax(-1.0, 0.5 * detB));
    const double phi = acos(r) / 3.0;
    return q + 2.0 * p * cos(phi + kTwoPi / 3.0);
}

__device__ __forceinline__ double det3(const double M[3][3]) {
    return M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
           M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
}

__device__ __forceinline__ void inv3(const double M[3][3], double R[3][3]) {
    const double d = 1.0 / det3(M);
    R[0][0] = (M[1][1] * M[2][2] - M[1][2] * M[2][1]) * d;
    R[0][1] = (M[0][2] * M[2][1] - M[0][1] * M[2][2]) * d;
    R[0][2] = (M[0][1] * M[1][2] - M[0][2] * M[1][1]) * d;
    R[1][0] = (M[1][2] * M[2][0] - M[1][0] * M[2][2]) * d;
    R[1][1] = (M[0][0] * M[2][2] - M[0][2] * M[2][0]) * d;
    R[1][2] = (M[0][2] * M[1][0] - M[0][0] * M[1][2]) * d;
    R[2][0] = (M[1][0] * M[2][1] - M[1][1] * M[2][0]) * d;
    R[2][1] = (M[0][1] * M[2][0] - M[0][0] * M[2][1]) * d;
    R[2][2] = (M[0][0] * M[1][1] - M[0][1] * M[1][0]) * d;
}

// Equilibrium record and primitive output from the converged parameters.
__device__ void write_point(const NewtonArgs &A, int64_t pt, double rho, const double U[3], double th,
                            const double Am[3][3], const double z[5], double inv_tau, double res) {
    double Ai[3][3];
    inv3(Am, Ai);
    double m[3], mAm = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) m[i] = (Ai[i][0] * z[1] + Ai[i][1] * z[2] + Ai[i][2] * z[3]) / z[4];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) mAm += m[i] * Am[i][j] * m[j];
    const double st = sqrt(th);
    double *eq = A.eq + pt * kEqW;
    eq[EQ_C0] = log(rho) - 1.5 * log(th) + z[0] + 0.5 * z[4] * mAm;
#pragma unroll
    for (int d = 0; d < 3; ++d) eq[EQ_V + d] = U[d] + st * m[d];
    const double sc = z[4] / th;
    eq[EQ_B] = sc * Am[0][0]; eq[EQ_B + 1] = sc * Am[1][1]; eq[EQ_B + 2] = sc * Am[2][2];
    eq[EQ_B + 3] = sc * Am[0][1]; eq[EQ_B + 4] = sc * Am[0][2]; eq[EQ_B + 5] = sc * Am[1][2];
    eq[EQ_INVTAU] = inv_tau;
    eq[EQ_RES] = res;
    double *pp = A.prim + pt * 5;
    pp[0] = rho * exp(z[0] + 0.5 * z[4] * mAm) * pow(kTwoPi / z[4], 1.5) / sqrt(det3(Am));
#pragma unroll
    for (int d = 0; d < 3; ++d) pp[1 + d] = eq[EQ_V + d];
    pp[4] = th / z[4];
#pragma unroll
    for (int a = 0; a < 5; ++a) A.z[pt * 5 + a] = z[a];
}

__device__ void write_nonreal(const NewtonArgs &A, int64_t pt) {
    double *eq = A.eq + pt * kEqW;
    eq[EQ_C0] = -INFINITY;
    for (int a = 1; a < kEqW; ++a) eq[a] = 0.0;
    for (int a = 0; a < 5; ++a) { A.prim[pt * 5 + a] = 0.0; A.z[pt * 5 + a] = 0.0; }
}

// Per-point outcome; the counters are aggregated afterwards by k_stats_reduce
// (per-point atomics on a handful of counters would serialise the kernel).
__device__ void record_stats(const NewtonArgs &A, int64_t pt, int iters, int evals, int status, double res) {
    if (A.pt_iters) A.pt_iters[pt] = iters;
    if (A.pt_evals) A.pt_evals[pt] = evals;
    if (A.pt_status) A.pt_status[pt] = status;
    if (A.pt_resid) A.pt_resid[pt] = res;
}

// Histogram of iterations, fallback / ES-guard counts, total evaluations and
// the largest final residual, aggregated per workgroup in LDS and then added
// to the handle's counters with one atomic per non-empty bin.
__global__ __launch_bounds__(256) void k_stats_reduce(int64_t npts, const int32_t *__restrict__ iters,
                                                      const int32_t *__restrict__ evals,
                                                      const int32_t *__restrict__ status,
                                                      const double *__restrict__ resid, unsigned long long *stats,
                                                      unsigned long long *maxres) {
    __shared__ unsigned int hist[kHist + 3];
    __shared__ double rmax[256];
    for (int i = threadIdx.x; i < kHist + 3; i += 256) hist[i] = 0u;
    __syncthreads();
    double m = 0.0;
    for (int64_t pt = (int64_t)blockIdx.x * 256 + threadIdx.x; pt < npts; pt += (int64_t)gridDim.x * 256) {
        const int it = iters[pt];
        atomicAdd(&hist[it < kHist ? (it < 0 ? 0 : it) : kHist - 1], 1u);
        if (status[pt] == FR_DVM_NEWTON_FALLBACK) atomicAdd(&hist[kHist], 1u);
        if (status[pt] == FR_DVM_NEWTON_ESGUARD) atomicAdd(&hist[kHist + 1], 1u);
        atomicAdd(&hist[kHist + 2], (unsigned int)evals[pt]);
        const double r = resid[pt];
        if (r >= 0.0 && isfinite(r)) m = fmax(m, r);
    }
    rmax[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) rmax[threadIdx.x] = fmax(rmax[threadIdx.x], rmax[threadIdx.x + o]);
        __syncthreads();
    }
    for (int i = threadIdx.x; i < kHist + 3; i += 256)
        if (hist[i]) atomicAdd(&stats[i], (unsigned long long)hist[i]);
    if (threadIdx.x == 0 && rmax[0] > 0.0) atomicMax(maxres, (unsigned long long)__double_as_longlong(rmax[0]));
}

// Second starting point besides the cold one (warm or learned), if any.
__device__ bool alt_start(const NewtonArgs &A, int64_t pt, const double zc[5], double z[5]) {
    bool ok = false;
    if (A.guess == FR_DVM_GUESS_WARM) {
        ok = true;
#pragma unroll
        for (int a = 0; a < 5; ++a) { z[a] = A.z[pt * 5 + a]; ok = ok && isfinite(z[a]); }
    } else if (A.guess == FR_DVM_GUESS_MLP && A.dz_guess) {
        ok = true;
#pragma unroll
        for (int a = 0; a < 5; ++a) { z[a] = zc[a] + (double)A.dz_guess[pt * 5 + a]; ok = ok && isfinite(z[a]); }
    }
    return ok && z[4] > 0.0;
}

// Residual rows psi = (1, c, |c|^2/2) against the targets (1, 0, 0, 0, 3/2).
__device__ __forceinline__ void residual(const Sums &s, double r[5]) {
    r[0] = s.S0 - 1.0;
    r[1] = s.Sc[0];
    r[2] = s.Sc[1];
    r[3] = s.Sc[2];
    r[4] = 0.5 * (s.Scc[0] + s.Scc[1] + s.Scc[2]) - 1.5;
}

// Below this residual norm the iteration keeps its Jacobian (chord steps)
// and evaluates only the residual sums; from a start this close the chord
// contraction factor is of the order of the distance to the root.
constexpr double kChord = 1e-5;

// Damped Newton from the better of the cold start and the alternative start.
// Returns 1 on convergence; z, res, iterations (linear solves) and evals
// (sum passes) are outputs.
template <typename SumsFn>
__device__ int newton_solve(const NewtonArgs &A, SumsFn sums, int64_t pt, const double zc[5], double z[5],
                            double &res, int &iters, int &evals) {
    // s: full sums at the point of the current Jacobian (assembled right
    // before each solve, to keep register pressure low); r: residual at z.
    double r[5], J[5][5];
    Sums s;
    // the alternative start is tried first; the cold start is evaluated too
    // only when the alternative is not already close (scaled residual > 1e-2)
    const bool have_alt = A.guess != FR_DVM_GUESS_COLD && alt_start(A, pt, zc, z);
    if (!have_alt) {
#pragma unroll
        for (int a = 0; a < 5; ++a) z[a] = zc[a];
    }
    sums(z, s, true);
    residual(s, r);
    evals = 1;
    if (have_alt && !(norm2_5(r) <= 1e-2)) {
        Sums sc;
        double rc[5];
        sums(zc, sc, true);
        residual(sc, rc);
        ++evals;
        if (!(norm2_5(r) <= norm2_5(rc))) {
            s = sc;
#pragma unroll
            for (int a = 0; a < 5; ++a) { z[a] = zc[a]; r[a] = rc[a]; }
        }
    }
    int conv = 0, it, rej = 0;  // rej: rejected line-search trials over the whole solve
    for (it = 0; it < A.max_iter; ++it) {
        const double rn = norm2_5(r), ri = normi_5(r);
        double rhs[5] = {-r[0], -r[1], -r[2], -r[3], -r[4]}, dz[5], rdum[5];
        assemble(s, rdum, J);
        const bool ok = solve5(J, rhs, dz);
        if (ok && ri <= A.tol) {
            // converged: one extra step makes the result path independent
#pragma unroll
            for (int a = 0; a < 5; ++a) z[a] += dz[a];
            res = ri;
            conv = 1;
            ++it;
            break;
        }
        if (!ok) break;
        const bool chord = rn <= kChord;
        double alpha = 1.0, zt[5], rt[5];
        Sums st;
        bool acc = false;
        while (rej < kRejectBudget) {
#pragma unroll
            for (int a = 0; a < 5; ++a) zt[a] = z[a] + alpha * dz[a];
            if (zt[4] > 0.0) {
                sums(zt, st, !chord);
                ++evals;
                residual(st, rt);
                if (norm2_5(rt) < (1.0 - 1e-4 * alpha) * rn) { acc = true; break; }
            }
            alpha *= 0.5;
            ++rej;
        }
        if (!acc) {
            // stagnation at the rounding floor of the FP64 sums
            if (ri <= 100.0 * A.tol) { res = ri; conv = 1; ++it; }
            break;
        }
#pragma unroll
        for (int a = 0; a < 5; ++a) { z[a] = zt[a]; r[a] = rt[a]; }
        if (!chord) {
            s = st;
        } else if (norm2_5(rt) > 1e-2 * rn) {
            // slow chord contraction: refresh the Jacobian at the new point
            sums(z, s, true);
            ++evals;
            residual(s, r);
        }
    }
    iters = it;
    if (!conv) {
        res = normi_5(r);
#pragma unroll
        for (int a = 0; a < 5; ++a) z[a] = zc[a];
    }
    return conv;
}

// The same iteration as newton_solve, written as one loop around a single
// evaluation of the sums: the two points of a wave evaluate together in
// whatever phase each is (start, cold start, line-search trial, Jacobian
// refresh), and the sums code is emitted once.  The sums at the current
// Jacobian (s) and at the point under evaluation (st) are held by the
// caller, in LDS, and so is the iteration's state: the start zc, the iterate
// z, the point under evaluation ze, its residual r and the step dz (the
// sums need most of the register file).
template <typename SumsFn>
__device__ int newton_solve_es(const NewtonArgs &A, SumsFn sums, int64_t pt, const double *zc, double *z,
                               double *ze, double *r, double *dz, Sums &s, Sums &st, double &res, int &iters,
                               int &evals) {
    enum { kStart, kCold, kTrial, kRefresh };
    double za[5];
    const bool have_alt = A.guess != FR_DVM_GUESS_COLD && alt_start(A, pt, zc, za);
#pragma unroll
    for (int a = 0; a < 5; ++a) z[a] = have_alt ? za[a] : zc[a];
#pragma unroll
    for (int a = 0; a < 5; ++a) { ze[a] = z[a]; r[a] = 0.0; dz[a] = 0.0; }
    int phase = kStart, it = 0, hh = 0, conv = 0;
    bool jac = true, chord = false;
    double alpha = 1.0, rn = 0.0, ri = 0.0;
    evals = 0;
    for (;;) {
        Sums &tg = (phase == kStart || phase == kRefresh) ? s : st;
        sums(ze, tg, jac);
        ++evals;
        double re[5];
        residual(tg, re);
        if (phase == kStart) {
#pragma unroll
            for (int a = 0; a < 5; ++a) r[a] = re[a];
            if (have_alt && !(norm2_5(r) <= 1e-2)) {
                // the alternative start is not already close: evaluate the
                // cold start too and keep the better one
                phase = kCold;
#pragma unroll
                for (int a = 0; a < 5; ++a) ze[a] = zc[a];
                continue;
            }
        } else if (phase == kCold) {
            if (!(norm2_5(r) <= norm2_5(re))) {
                s = st;
#pragma unroll
                for (int a = 0; a < 5; ++a) { z[a] = zc[a]; r[a] = re[a]; }
            }
        } else if (phase == kTrial) {
            const double rt = norm2_5(re);
            if (rt < (1.0 - 1e-4 * alpha) * rn) {
#pragma unroll
                for (int a = 0; a < 5; ++a) { z[a] = ze[a]; r[a] = re[a]; }
                if (!chord) {
                    s = st;
                } else if (rt > 1e-2 * rn) {
                    // slow chord contraction: refresh the Jacobian at z (= ze)
                    phase = kRefresh;
                    jac = true;
                    continue;
                }
                ++it;
            } else {
                // rejected: halve the step until the trial is admissible
                do {
                    alpha *= 0.5;
                    ++hh;
#pragma unroll
                    for (int a = 0; a < 5; ++a) ze[a] = z[a] + alpha * dz[a];
                } while (hh < kRejectBudget && !(ze[4] > 0.0));
                if (hh < kRejectBudget) continue;
                // stagnation at the rounding floor of the FP64 sums
                if (ri <= 100.0 * A.tol) { res = ri; conv = 1; ++it; }
                break;
            }
        } else {  // kRefresh
#pragma unroll
            for (int a = 0; a < 5; ++a) r[a] = re[a];
            ++it;
        }
        // Newton step from z with the Jacobian of s
        if (it >= A.max_iter) break;
        rn = norm2_5(r);
        ri = normi_5(r);
        double J[5][5], rdum[5];
        double rhs[5] = {-r[0], -r[1], -r[2], -r[3], -r[4]};
        assemble(s, rdum, J);
        const bool ok = solve5(J, rhs, dz);
        if (ok && ri <= A.tol) {
            // converged: one extra step makes the result path independent
#pragma unroll
            for (int a = 0; a < 5; ++a) z[a] += dz[a];
            res = ri;
            conv = 1;
            ++it;
            break;
        }
        if (!ok) break;
        chord = rn <= kChord;
        alpha = 1.0;
        // hh counts the rejected trials of the whole solve (not reset here)
#pragma unroll
        for (int a = 0; a < 5; ++a) ze[a] = z[a] + alpha * dz[a];
        while (hh < kRejectBudget && !(ze[4] > 0.0)) {
            alpha *= 0.5;
            ++hh;
#pragma unroll
            for (int a = 0; a < 5; ++a) ze[a] = z[a] + alpha * dz[a];
        }
        if (hh >= kRejectBudget) {
            if (ri <= 100.0 * A.tol) { res = ri; conv = 1; ++it; }
            break;
        }
        phase = kTrial;
        jac = !chord;
    }
    iters = it;
    if (!conv) {
        res = normi_5(r);
#pragma unroll
        for (int a = 0; a < 5; ++a) z[a] = zc[a];
    }
    return conv;
}

__global__ __launch_bounds__(256) void k_newton_bgk(const NewtonArgs A) {
    const int64_t pt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pt >= A.npts) return;
    const double *Q = A.Q + pt * A.nmom;
    const double rho = Q[0];
    const double irho = 1.0 / rho;
    double U[3] = {Q[1] * irho, Q[2] * irho, Q[3] * irho};
    // E - rho |U|^2 / 2 = (3 + delta)/2 rho theta
    const double E = record_energy(Q, A.nmom);
    const double th = (2.0 / (3.0 + A.delta)) * (E * irho - 0.5 * (U[0] * U[0] + U[1] * U[1] + U[2] * U[2]));
    if (!(rho > 0.0) || !(th > 0.0) || !isfinite(rho) || !isfinite(th)) {
        write_nonreal(A, pt);
        if (A.gfp) A.gfp[pt] = 0.0;
        record_stats(A, pt, 0, 0, FR_DVM_NEWTON_NONREAL, -1.0);
        return;
    }
    if (A.gfp) A.gfp[pt] = 0.5 * A.delta * th;
    const double inv_tau = rho * th / viscosity(A, th);
    const double ist = 1.0 / sqrt(th);
    const double zc[5] = {-1.5 * log(kTwoPi), 0.0, 0.0, 0.0, 1.0};
    double z[5];
    auto fn = [&](const double zz[5], Sums &s, bool) { sums_bgk(A, U, ist, zz, s); };
    double res;
    int iters, evals;
    const int conv = newton_solve(A, fn, pt, zc, z, res, iters, evals);
    const double Am[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    write_point(A, pt, rho, U, th, Am, z, inv_tau, res);
    record_stats(A, pt, iters, evals, conv ? FR_DVM_NEWTON_OK : FR_DVM_NEWTON_FALLBACK, res);
}

#ifndef FRDVM_WAVES_ES
#define FRDVM_WAVES_ES 3
#endif
// One solution point per kLpp lanes: two per wave, four per 128-thread
// workgroup (about 6 KB of LDS per point at 20^3 velocities, so LDS admits
// six workgroups per CU and registers decide the occupancy).
constexpr int kEsBlock = 128;
constexpr int kEsPts = kEsBlock / kLpp;
constexpr int kSumsD = (int)(sizeof(Sums) / sizeof(double));
constexpr int kStateD = 38;  // U[3], A[3][3], zc, z, ze, r, dz [5] each, pad

// LDS doubles per point of k_newton_es: two sum sets, the iteration state,
// then the factor tables.
__host__ __device__ inline int es_slot_doubles(const VGrid &vg, int use_fact) {
    return 2 * kSumsD + kStateD + (use_fact ? fact_layout(vg).total : 0);
}

__global__ __launch_bounds__(kEsBlock) __attribute__((amdgpu_waves_per_eu(FRDVM_WAVES_ES))) void k_newton_es(
    const NewtonArgs A) {
    const int lane = threadIdx.x % kLpp;
    const int slot = threadIdx.x / kLpp;
    const int64_t pt = (int64_t)blockIdx.x * kEsPts + slot;
    if (pt >= A.npts) return;  // a point's lanes exit together
    const double *Q = A.Q + pt * A.nmom;
    const double rho = Q[0];
    const double irho = 1.0 / rho;
    double U[3] = {Q[1] * irho, Q[2] * irho, Q[3] * irho};
    // raw second moments -> pressure tensor Pi = M2 - rho U U^T
    const double Pi[6] = {Q[4] - rho * U[0] * U[0], Q[5] - rho * U[1] * U[1], Q[6] - rho * U[2] * U[2],
                          Q[7] - rho * U[0] * U[1], Q[8] - rho * U[0] * U[2], Q[9] - rho * U[1] * U[2]};
    // (3 + delta) rho theta = tr Pi + 2 (integral of G)
    const double th = (Pi[0] + Pi[1] + Pi[2] + (A.nmom == 11 ? 2.0 * Q[10] : 0.0)) / ((3.0 + A.delta) * rho);
    if (!(rho > 0.0) || !(th > 0.0) || !isfinite(rho) || !isfinite(th)) {
        if (lane == 0) {
            write_nonreal(A, pt);
            if (A.gfp) A.gfp[pt] = 0.0;
            record_stats(A, pt, 0, 0, FR_DVM_NEWTON_NONREAL, -1.0);
        }
        return;
    }
    if (A.gfp && lane == 0) A.gfp[pt] = 0.5 * A.delta * th;
    const double Pr = A.Pr;
    const double inv_tau = Pr * rho * th / viscosity(A, th);
    const double ist = 1.0 / sqrt(th);
    double Am[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    int status = FR_DVM_NEWTON_OK;
    {
        const double a1 = th / Pr, a2 = (1.0 - 1.0 / Pr) * irho;
        const double T[3][3] = {{a1 + a2 * Pi[0], a2 * Pi[3], a2 * Pi[4]},
                                {a2 * Pi[3], a1 + a2 * Pi[1], a2 * Pi[5]},
                                {a2 * Pi[4], a2 * Pi[5], a1 + a2 * Pi[2]}};
        if (sym3_min_eig(T) <= 1e-8 * th) {
            status = FR_DVM_NEWTON_ESGUARD;
        } else {
            double Ti[3][3];
            inv3(T, Ti);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) Am[i][j] = th * Ti[i][j];
        }
    }
    const double zc[5] = {-1.5 * log(kTwoPi) + 0.5 * log(det3(Am)), 0.0, 0.0, 0.0, 1.0};
    double z[5];
    const double wscale = ist * ist * ist;
    // per point: the two sum sets of the iteration, the iteration state and
    // the point's frame (U, A), then the factor tables
    extern __shared__ double es_lds[];
    double *sl = es_lds + slot * es_slot_doubles(A.vg, A.use_fact);
    Sums &s_cur = *reinterpret_cast<Sums *>(sl);
    Sums &s_try = *reinterpret_cast<Sums *>(sl + kSumsD);
    double *ns = sl + 2 * kSumsD;
    double *Us = ns, *zcs = ns + 12, *zs = ns + 17, *zes = ns + 22, *rs = ns + 27, *dzs = ns + 32;
    double(*Ams)[3] = reinterpret_cast<double(*)[3]>(ns + 3);
    double *tb = ns + kStateD;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        Us[d] = U[d];
#pragma unroll
        for (int b = 0; b < 3; ++b) Ams[d][b] = Am[d][b];
    }
#pragma unroll
    for (int a = 0; a < 5; ++a) zcs[a] = zc[a];
    auto fn = [&](const double *zz, Sums &s, bool jac) {
        if (!(A.use_fact && sums_es_fact(A, lane, tb, Us, ist, Ams, zz, s, jac)))
            sums_es(A, lane, Us, ist, wscale, Ams, zz, s, jac);
    };
    double res;
    int iters, evals;
    const int conv = newton_solve_es(A, fn, pt, zcs, zs, zes, rs, dzs, s_cur, s_try, res, iters, evals);
    if (lane == 0) {
        write_point(A, pt, rho, Us, th, Ams, zs, inv_tau, res);
        record_stats(A, pt, iters, evals, conv ? status : FR_DVM_NEWTON_FALLBACK, res);
    }
}

// Size of the discrete-velocity error of the continuous equilibrium, which
// scales the learned correction: trapezoid aliasing exp(-2 pi^2 theta/du^2)
// plus truncation by the velocity box exp(-(u_max - |U_d|)^2 / (2 theta)).
__device__ __forceinline__ double guess_envelope(const double U[3], double th, double umax, double du) {
    double tr = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double g = fmax(umax - fabs(U[d]), 0.0);
        tr = fmax(tr, exp(-g * g / (2.0 * th)));
    }
    const double s = exp(-0.5 * kTwoPi * kTwoPi * th / (du * du)) + tr;
    return fmin(fmax(s, 1e-10), 1.0);  // below 1e-10 the correction is Newton round-off
}

__global__ void k_mlp_scale(int64_t n, const float *__restrict__ env, float *__restrict__ dz) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n * 5) dz[i] *= env[i / 5];
}

// Features of the learned guess from the moments: [ln rho, U/u_max, ln theta,
// u_max/10, n_v/32, sin and cos of the grid phase 2 pi (U - umin)/du] (FP32)
// and the correction envelope; non-realizable
// points get zeros (Newton marks them).
__global__ void k_mlp_features(int64_t npts, int nmom, const double *__restrict__ Q, const VGrid vg, double umax,
                               double du, float *__restrict__ X, float *__restrict__ env) {
    const int64_t pt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pt >= npts) return;
    const double *q = Q + pt * nmom;
    const double rho = q[0];
    const double U[3] = {q[1] / rho, q[2] / rho, q[3] / rho};
    const double E = nmom == 5 ? q[4] : 0.5 * (q[4] + q[5] + q[6]);
    const double th = (2.0 / 3.0) * (E / rho - 0.5 * (U[0] * U[0] + U[1] * U[1] + U[2] * U[2]));
    float *x = X + pt * FR_MLP_INPUTS;
    if (!(rho > 0.0) || !(th > 0.0)) {
        for (int a = 0; a < FR_MLP_INPUTS; ++a) x[a] = 0.f;
        env[pt] = 0.f;
        return;
    }
    env[pt] = (float)guess_envelope(U, th, umax, du);
    x[0] = (float)log(rho);
    x[1] = (float)(U[0] / umax);
    x[2] = (float)(U[1] / umax);
    x[3] = (float)(U[2] / umax);
    x[4] = (float)log(th);
    x[5] = (float)(umax / 10.0);
    x[6] = (float)(vg.nv[0] / 32.0);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double ph = vg.du[d] > 0.0 ? kTwoPi * (U[d] - vg.umin[d]) / vg.du[d] : 0.0;
        x[7 + d] = (float)sin(ph);
        x[10 + d] = (float)cos(ph);
    }
}

__global__ void k_collide(const VGrid vg, const double *__restrict__ eqs, const void *fv, void *Sv, int accumulate,
                          int fp64, int ncomp, const double *__restrict__ gfp) {
    const int64_t pt = blockIdx.x;
    const double *eqp = eqs + pt * kEqW;
    double eq[kEqW];
#pragma unroll
    for (int a = 0; a < kEqW; ++a) eq[a] = eqp[a];
    // the pair's G relaxes to delta theta / 2 times the equilibrium of F:
    // its exponent is shifted by the logarithm of that factor
    const double lg = ncomp == 2 ? (gfp[pt] > 0.0 ? log(gfp[pt]) : -1000.0) : 0.0;
    const int nut = vg.nu * ncomp;
    for (int kk = threadIdx.x; kk < nut; kk += blockDim.x) {
        const int comp = kk >= vg.nu, k = kk - comp * vg.nu;
        const int i = k % vg.nv[0], j = (k / vg.nv[0]) % vg.nv[1], l = k / (vg.nv[0] * vg.nv[1]);
        const double u[3] = {gridu(vg, 0, i), gridu(vg, 1, j), gridu(vg, 2, l)};
        const int64_t idx = pt * nut + kk;
        const double c0g = eq[EQ_C0] + (comp ? lg : 0.0);
        if (fp64) {
            const double c0 = u[0] - eq[EQ_V], c1 = u[1] - eq[EQ_V + 1], c2 = u[2] - eq[EQ_V + 2];
            const double q = eq[EQ_B] * c0 * c0 + eq[EQ_B + 1] * c1 * c1 + eq[EQ_B + 2] * c2 * c2 +
                             2.0 * (eq[EQ_B + 3] * c0 * c1 + eq[EQ_B + 4] * c0 * c2 + eq[EQ_B + 5] * c1 * c2);
            const double g = exp(c0g - 0.5 * q);
            const double f = ((const double *)fv)[idx];
            const double S = (g - f) * eq[EQ_INVTAU];
            double *So = (double *)Sv;
            So[idx] = accumulate ? So[idx] + S : S;
        } else {
            // the exponent in FP64 and the exponential rounded once to FP32,
            // as in the fused stage
            const double c0 = u[0] - eq[EQ_V], c1 = u[1] - eq[EQ_V + 1], c2 = u[2] - eq[EQ_V + 2];
            const double q = eq[EQ_B] * c0 * c0 + eq[EQ_B + 1] * c1 * c1 + eq[EQ_B + 2] * c2 * c2 +
                             2.0 * (eq[EQ_B + 3] * c0 * c1 + eq[EQ_B + 4] * c0 * c2 + eq[EQ_B + 5] * c1 * c2);
            const float g = exp_to_f32(c0g - 0.5 * q);
            const float f = ((const float *)fv)[idx];
            const float S = (g - f) * (float)eq[EQ_INVTAU];
            float *So = (float *)Sv;
            So[idx] = accumulate ? So[idx] + S : S;
        }
    }
}

__global__ void k_moments_out(int64_t npts, int nmom, const double *__restrict__ Q, double *__restrict__ out) {
    const int64_t pt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pt >= npts) return;
    const double *q = Q + pt * nmom;
    double *o = out + pt * 5;
    o[0] = q[0]; o[1] = q[1]; o[2] = q[2]; o[3] = q[3];
    o[4] = record_energy(q, nmom);
}

// Gradient-length local Knudsen number (Section "Results"):
// Kn = lambda |grad rho| / rho with the hard-sphere-type mean free path
// lambda = mu(theta)/rho sqrt(pi/(2 theta)).  grad rho is the derivative of
// the element's solution polynomial of rho (the FR interpolant, no interface
// correction); on an axis-aligned box d/dx_d = (2/h_d) d/dxi_d, on a general
// element grad = (1/|J|) sum_d a^d d/dxi_d.  One wave per
// element (ns <= 64 points), the density of the element staged in LDS.
// Points with rho <= 0 or theta <= 0 get 0.
constexpr int kKnElems = 4;

__global__ __launch_bounds__(64 * kKnElems) void k_kn_gll(NewtonArgs A, Ops1D ops, int n, int64_t ne,
                                                          const double *__restrict__ gfac, const double *__restrict__ S,
                                                          const double *__restrict__ ijac, double *__restrict__ kn) {
    __shared__ double srho[kKnElems][64];
    const int w = threadIdx.x >> 6, s = threadIdx.x & 63;
    const int64_t e = (int64_t)blockIdx.x * kKnElems + w;
    const int ns = n * n * n;
    const bool live = e < ne && s < ns;
    const int64_t pt = e * ns + s;
    if (live) srho[w][s] = A.Q[pt * A.nmom];
    __syncthreads();
    if (!live) return;
    const int i = s % n, j = (s / n) % n, l = s / (n * n);
    double d0 = 0, d1 = 0, d2 = 0;
    for (int m = 0; m < n; ++m) {
        d0 += ops.D[i * n + m] * srho[w][m + n * (j + n * l)];
        d1 += ops.D[j * n + m] * srho[w][i + n * (m + n * l)];
        d2 += ops.D[l * n + m] * srho[w][i + n * (j + n * m)];
    }
    if (S) {  // general element: grad = (1/|J|) sum_d a^d d/dxi_d
        const double *a = S + pt * 9;
        const double g0 = ijac[pt] * (a[0] * d0 + a[3] * d1 + a[6] * d2);
        const double g1 = ijac[pt] * (a[1] * d0 + a[4] * d1 + a[7] * d2);
        const double g2 = ijac[pt] * (a[2] * d0 + a[5] * d1 + a[8] * d2);
        d0 = g0;
        d1 = g1;
        d2 = g2;
    } else {
        d0 *= gfac[e * 3 + 0];
        d1 *= gfac[e * 3 + 1];
        d2 *= gfac[e * 3 + 2];
    }
    const double *q = A.Q + pt * A.nmom;
    const double rho = q[0];
    const double ux = q[1] / rho, uy = q[2] / rho, uz = q[3] / rho;
    const double E = record_energy(q, A.nmom);
    const double th = (2.0 / (3.0 + A.delta)) * (E / rho - 0.5 * (ux * ux + uy * uy + uz * uz));
    double out = 0.0;
    if (rho > 0.0 && th > 0.0) {
        const double lam = viscosity(A, th) / rho * sqrt(kTwoPi / (4.0 * th));
        out = lam * sqrt(d0 * d0 + d1 * d1 + d2 * d2) / rho;
    }
    kn[pt] = out;
}

// Domain totals: one workgroup, fixed-order strided sums and tree reduction.
__global__ __launch_bounds__(1024) void k_totals(int64_t npts, int nmom, const double *__restrict__ Q,
                                                 const double *__restrict__ wJ, double *__restrict__ out) {
    __shared__ double red[5][1024];
    double a[5] = {0, 0, 0, 0, 0};
    for (int64_t pt = threadIdx.x; pt < npts; pt += 1024) {
        const double *q = Q + pt * nmom;
        const double w = wJ[pt];
        a[0] += w * q[0]; a[1] += w * q[1]; a[2] += w * q[2]; a[3] += w * q[3];
        a[4] += w * record_energy(q, nmom);
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) red[c][threadIdx.x] = a[c];
    __syncthreads();
    for (int o = 512; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o)
#pragma unroll
            for (int c = 0; c < 5; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x < 5) out[threadIdx.x] = red[threadIdx.x][0];
}

int check(fr_dvm *h, const char *what) {
    hipError_t st = hipGetLastError();
    if (st != hipSuccess) return h->fail(FR_DVM_EHIP, std::string(what) + ": " + hipGetErrorString(st));
    return FR_DVM_OK;
}

NewtonArgs newton_args(fr_dvm *h, int guess) {
    NewtonArgs A;
    std::memset(&A, 0, sizeof(A));
    A.vg = h->vg;
    A.npts = h->ne * h->ns;
    A.nmom = h->nmom;
    A.wax = h->d_wax;
    A.Q = h->d_Q;
    A.eq = h->d_eq;
    A.z = h->d_z;
    A.prim = h->d_prim;
    A.stats = reinterpret_cast<unsigned long long *>(h->d_stats);
    A.maxres = reinterpret_cast<unsigned long long *>(h->d_maxres);
    A.Pr = h->prm.prandtl;
    A.mu_ref = h->prm.mu_ref;
    A.theta_ref = h->prm.theta_ref;
    A.omega = h->prm.omega;
    A.theta_s = h->prm.theta_s;
    A.visc_law = h->prm.visc_law;
    A.tol = h->prm.newton_tol;
    A.max_iter = h->prm.newton_max_iter;
    A.guess = (guess == FR_DVM_GUESS_WARM && !h->zvalid) ? FR_DVM_GUESS_COLD : guess;
    // the learned start is trained on monatomic states: cold start for the pair
    if (A.guess == FR_DVM_GUESS_MLP && (!h->d_mlp || h->ncomp == 2)) A.guess = FR_DVM_GUESS_COLD;
    A.delta = h->ncomp == 2 ? h->delta : 0.0;
    A.gfp = h->d_gfp;
    return A;
}

double grid_umax(const VGrid &vg) {
    double m = 0;
    for (int d = 0; d < 3; ++d)
        m = std::fmax(m, std::fmax(std::fabs(vg.umin[d]), std::fabs(vg.umin[d] + (vg.nv[d] - 1) * vg.du[d])));
    return m;
}

// Learned correction dz[n][5] (float) for moment vectors Q[n][nmom], batched
// through the MLP forward kernels.
int mlp_predict(fr_dvm *h, const double *Q, int64_t n, int nmom, float *dz) {
    const int64_t batch = 65536;
    const int64_t nb = n < batch ? n : batch;
    const size_t need_x = (size_t)nb * (FR_MLP_INPUTS + 1), need_w = fr_mlp_workspace_floats(h->mlp_hidden, nb);
    if (h->mlp_x_n < need_x || h->mlp_work_n < need_w) {
        if (h->d_mlp_x) (void)hipFree(h->d_mlp_x);
        if (h->d_mlp_work) (void)hipFree(h->d_mlp_work);
        h->d_mlp_x = nullptr;
        h->d_mlp_work = nullptr;
        if (hipMalloc(&h->d_mlp_x, need_x * sizeof(float)) != hipSuccess ||
            hipMalloc(&h->d_mlp_work, need_w * sizeof(float)) != hipSuccess)
            return h->fail(FR_DVM_ENOMEM, "MLP workspace");
        h->mlp_x_n = need_x;
        h->mlp_work_n = need_w;
    }
    const double umax = grid_umax(h->vg);
    const double du = std::fmax(h->vg.du[0], std::fmax(h->vg.du[1], h->vg.du[2]));
    float *env = h->d_mlp_x + (size_t)nb * FR_MLP_INPUTS;
    for (int64_t b0 = 0; b0 < n; b0 += batch) {
        const int64_t m = (n - b0) < batch ? (n - b0) : batch;
        hipLaunchKernelGGL(k_mlp_features, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, h->stream, m, nmom,
                           Q + b0 * nmom, h->vg, umax, du, h->d_mlp_x, env);
        int rc = fr_mlp_forward(h->mlp_hidden, h->d_mlp, h->d_mlp_x, m, dz + b0 * 5, h->d_mlp_work, h->stream);
        if (rc) return h->fail(rc, "MLP forward");
        hipLaunchKernelGGL(k_mlp_scale, dim3((unsigned)((m * 5 + 255) / 256)), dim3(256), 0, h->stream, m, env,
                           dz + b0 * 5);
    }
    return check(h, "MLP features");
}

int ensure_dz(fr_dvm *h, int64_t n) {
    if (h->dz_n >= (size_t)n) return FR_DVM_OK;
    if (h->d_mlp_dz) (void)hipFree(h->d_mlp_dz);
    h->d_mlp_dz = nullptr;
    if (hipMalloc(&h->d_mlp_dz, sizeof(float) * 5 * n) != hipSuccess) return h->fail(FR_DVM_ENOMEM, "MLP output");
    h->dz_n = n;
    return FR_DVM_OK;
}

}  // namespace

namespace {

// The Newton kernel and its statistics over the points [p0, p0 + np) on
// stream s: every per-point array of A is offset to p0, so the kernels see a
// contiguous range starting at their point 0.
int newton_run(fr_dvm *h, NewtonArgs A, int64_t p0, int64_t np, hipStream_t s) {
    A.npts = np;
    A.Q += p0 * A.nmom;
    A.eq += p0 * kEqW;
    A.z += p0 * 5;
    A.prim += p0 * 5;
    if (A.dz_guess) A.dz_guess += p0 * 5;
    if (A.gfp) A.gfp += p0;
    A.pt_iters = h->d_pt_iters + p0;
    A.pt_evals = h->d_pt_evals + p0;
    A.pt_status = h->d_pt_status + p0;
    A.pt_resid = h->d_pt_resid + p0;
    ProfScope ps(h, 1, s);
    if (h->prm.model == FR_DVM_ESBGK) {
        A.use_fact = (kEsPts * sizeof(double) * (size_t)es_slot_doubles(h->vg, 1) <= 65536) && !h->es_direct;
        const size_t shm = kEsPts * sizeof(double) * (size_t)es_slot_doubles(h->vg, A.use_fact);
        hipLaunchKernelGGL(k_newton_es, dim3((unsigned)((A.npts + kEsPts - 1) / kEsPts)), dim3(kEsBlock), shm, s, A);
    } else {
        hipLaunchKernelGGL(k_newton_bgk, dim3((unsigned)((A.npts + 255) / 256)), dim3(256), 0, s, A);
    }
    int64_t nb = (A.npts + 256 * 16 - 1) / (256 * 16);
    if (nb > 1024) nb = 1024;
    hipLaunchKernelGGL(k_stats_reduce, dim3((unsigned)nb), dim3(256), 0, s, A.npts, A.pt_iters, A.pt_evals,
                       A.pt_status, A.pt_resid, A.stats, A.maxres);
    const int rc = check(h, "newton kernel");
    if (!rc) h->newton_done = true;
    return rc;
}

}  // namespace

int launch_newton(fr_dvm *h, int guess) {
    // learned start where no previous solution exists, warm start afterwards
    if (guess == FR_DVM_GUESS_MLP_WARM) guess = h->zvalid ? FR_DVM_GUESS_WARM : FR_DVM_GUESS_MLP;
    NewtonArgs A = newton_args(h, guess);
    if (A.guess == FR_DVM_GUESS_MLP) {
        ProfScope ps(h, 3);
        int rc = ensure_dz(h, A.npts);
        if (!rc) rc = mlp_predict(h, h->d_Q, A.npts, h->nmom, h->d_mlp_dz);
        if (rc) return rc;
        A.dz_guess = h->d_mlp_dz;
    }
    const int rc = newton_run(h, A, 0, A.npts, h->stream);
    if (!rc) h->zvalid = 1;
    return rc;
}

int newton_part_ok(fr_dvm *h, int guess) {
    if (guess == FR_DVM_GUESS_MLP_WARM) guess = h->zvalid ? FR_DVM_GUESS_WARM : FR_DVM_GUESS_MLP;
    return newton_args(h, guess).guess != FR_DVM_GUESS_MLP;
}

int launch_newton_part(fr_dvm *h, int guess, int64_t p0, int64_t np, hipStream_t s) {
    if (guess == FR_DVM_GUESS_MLP_WARM) guess = h->zvalid ? FR_DVM_GUESS_WARM : FR_DVM_GUESS_MLP;
    NewtonArgs A = newton_args(h, guess);
    if (A.guess == FR_DVM_GUESS_MLP) return h->fail(FR_DVM_EINVAL, "learned start needs all points");
    if (p0 < 0 || np < 0 || p0 + np > A.npts) return h->fail(FR_DVM_EINVAL, "point range");
    return newton_run(h, A, p0, np, s);
}

// Newton on caller-supplied moment vectors (BGK form), for training targets
// and guess evaluation.  Scratch records are allocated per call.
int launch_newton_points(fr_dvm *h, const double *Q, int64_t n, int guess, double *z, int32_t *iters,
                         int32_t *evals, int32_t *status, double *resid) {
    if (n <= 0) return FR_DVM_OK;
    if (guess == FR_DVM_GUESS_MLP && !h->d_mlp) return h->fail(FR_DVM_EINVAL, "no MLP weights set");
    NewtonArgs A = newton_args(h, guess == FR_DVM_GUESS_MLP ? FR_DVM_GUESS_MLP : FR_DVM_GUESS_COLD);
    double *eq = nullptr, *prim = nullptr, *zz = nullptr;
    if (hipMalloc(&eq, sizeof(double) * kEqW * n) != hipSuccess || hipMalloc(&prim, sizeof(double) * 5 * n) != hipSuccess ||
        (!z && hipMalloc(&zz, sizeof(double) * 5 * n) != hipSuccess)) {
        if (eq) (void)hipFree(eq);
        if (prim) (void)hipFree(prim);
        return h->fail(FR_DVM_ENOMEM, "equilibrium scratch");
    }
    int rc = FR_DVM_OK;
    if (A.guess == FR_DVM_GUESS_MLP) {
        rc = ensure_dz(h, n);
        if (!rc) rc = mlp_predict(h, Q, n, 5, h->d_mlp_dz);
        A.dz_guess = h->d_mlp_dz;
    }
    if (!rc) {
        A.npts = n;
        A.nmom = 5;
        A.Q = Q;
        A.eq = eq;
        A.prim = prim;
        A.z = z ? z : zz;
        A.pt_iters = iters;
        A.pt_evals = evals;
        A.pt_status = status;
        A.pt_resid = resid;
        A.delta = 0.0;  // monatomic moment vectors
        A.gfp = nullptr;
        if (!(A.mu_ref > 0)) A.mu_ref = 1.0;  // tau is not an output here
        hipLaunchKernelGGL(k_newton_bgk, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, h->stream, A);
        rc = check(h, "newton kernel");
    }
    (void)hipStreamSynchronize(h->stream);
    (void)hipFree(eq);
    (void)hipFree(prim);
    if (zz) (void)hipFree(zz);
    return rc;
}

int launch_collide(fr_dvm *h, const void *f, void *S, int accumulate) {
    hipLaunchKernelGGL(k_collide, dim3((unsigned)(h->ne * h->ns)), dim3(256), 0, h->stream, h->vg, h->d_eq, f, S,
                       accumulate, h->prm.precision == FR_DVM_FP64 ? 1 : 0, h->ncomp, h->d_gfp);
    return check(h, "collide kernel");
}

int launch_prim_out(fr_dvm *h, double *Qp) {
    if (hipMemcpyAsync(Qp, h->d_prim, sizeof(double) * 5 * h->ne * h->ns, hipMemcpyDeviceToDevice, h->stream) !=
        hipSuccess)
        return h->fail(FR_DVM_EHIP, "copy of Q'");
    return FR_DVM_OK;
}

int launch_moments_out(fr_dvm *h, double *Q) {
    const int64_t npts = h->ne * h->ns;
    hipLaunchKernelGGL(k_moments_out, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, h->stream, npts, h->nmom,
                       h->d_Q, Q);
    return check(h, "moments output kernel");
}

int launch_kn_gll(fr_dvm *h, double *kn) {
    NewtonArgs A = newton_args(h, FR_DVM_GUESS_COLD);
    hipLaunchKernelGGL(k_kn_gll, dim3((unsigned)((h->ne + kKnElems - 1) / kKnElems)), dim3(64 * kKnElems), 0,
                       h->stream, A, h->ops, h->n, h->ne, h->axis_mode ? h->d_gfac : nullptr,
                       h->axis_mode ? nullptr : h->d_S, h->d_ijac, kn);
    return check(h, "Knudsen number kernel");
}

int launch_totals(fr_dvm *h, double *host_tot) {
    const int64_t npts = h->ne * h->ns;
    hipLaunchKernelGGL(k_totals, dim3(1), dim3(1024), 0, h->stream, npts, h->nmom, h->d_Q, h->d_wq3J, h->d_tot);
    int rc = check(h, "totals kernel");
    if (rc) return rc;
    if (hipMemcpyAsync(host_tot, h->d_tot, 5 * sizeof(double), hipMemcpyDeviceToHost, h->stream) != hipSuccess)
        return h->fail(FR_DVM_EHIP, "totals copy");
    if (hipStreamSynchronize(h->stream) != hipSuccess) return h->fail(FR_DVM_EHIP, "stream synchronise");
    return FR_DVM_OK;
}

}  // namespace frdvm
