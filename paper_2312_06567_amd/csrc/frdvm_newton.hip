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
// c = (u - U)/sqrt(theta) with weights w theta^-3/2 the five equations
// are sum_k wt_k (1, c_k, |c_k|^2/2) exp(z0 + z.c_k - z4 q(c_k)/2) =
// (1, 0, 0, 0, 3/2), q = |c|^2 (BGK) or c^T A c with A = theta T^-1 (ES-BGK).
//
// BGK kernel: one thread per point.  On a tensor velocity grid the BGK
// exponential factorises per axis, so each Newton iteration costs 3 n_v
// exponentials and 1-D power sums instead of n_v^3 terms.
// ES kernel: one wave64 per point, lanes over velocity nodes, butterfly
// reduction of the 17 sums (lane-symmetric: every lane gets the same bits).
#include <hip/hip_runtime.h>

#include <cmath>

#include "frdvm_common.h"

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
    int model;
    double Pr, mu_ref, theta_ref, omega, theta_s;
    int visc_law;
    double tol;
    int max_iter;
    int guess;
    const float *mlp;
    int mlp_hidden;
};

constexpr double kTwoPi = 6.283185307179586476925286766559;

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

// Gaussian elimination with partial pivoting on a 5x5 system (copies J).
__device__ bool solve5(const double J[5][5], const double b[5], double x[5]) {
    double M[5][6];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
#pragma unroll
        for (int j = 0; j < 5; ++j) M[i][j] = J[i][j];
        M[i][5] = b[i];
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        int piv = c;
        double best = fabs(M[c][c]);
#pragma unroll
        for (int r = c + 1; r < 5; ++r)
            if (fabs(M[r][c]) > best) { best = fabs(M[r][c]); piv = r; }
        if (!(best > 0.0)) return false;
#pragma unroll
        for (int r = c; r < 5; ++r) {
            if (r == piv && piv != c) {
#pragma unroll
                for (int j = 0; j < 6; ++j) { double t = M[c][j]; M[c][j] = M[r][j]; M[r][j] = t; }
            }
        }
#pragma unroll
        for (int r = c + 1; r < 5; ++r) {
            double fct = M[r][c] / M[c][c];
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
    return true;
}

__device__ double norm2_5(const double r[5]) {
    return sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3] + r[4] * r[4]);
}
__device__ double normi_5(const double r[5]) {
    double m = 0;
#pragma unroll
    for (int a = 0; a < 5; ++a) m = fmax(m, fabs(r[a]));
    return m;
}

// Assemble residual and Jacobian from the raw sums
//   S0 = sum wt e, Sc_i = sum wt c_i e, Scc (xx yy zz xy xz yz), Sq = sum wt q e,
//   Scq_i = sum wt c_i q e, Sc2c_i = sum wt |c|^2 c_i e, Sc2q = sum wt |c|^2 q e.
// Rows psi = (1, c, |c|^2/2), columns d/dz = (1, c, -q/2).
struct Sums {
    double S0, Sc[3], Scc[6], Sq, Scq[3], Sc2c[3], Sc2q;
};

__device__ void assemble(const Sums &s, double r[5], double J[5][5]) {
    const int ij[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
    double c2 = s.Scc[0] + s.Scc[1] + s.Scc[2];
    r[0] = s.S0 - 1.0;
    r[1] = s.Sc[0];
    r[2] = s.Sc[1];
    r[3] = s.Sc[2];
    r[4] = 0.5 * c2 - 1.5;
    J[0][0] = s.S0;
    for (int j = 0; j < 3; ++j) J[0][1 + j] = s.Sc[j];
    J[0][4] = -0.5 * s.Sq;
    for (int i = 0; i < 3; ++i) {
        J[1 + i][0] = s.Sc[i];
        for (int j = 0; j < 3; ++j) J[1 + i][1 + j] = s.Scc[ij[i][j]];
        J[1 + i][4] = -0.5 * s.Scq[i];
    }
    J[4][0] = 0.5 * c2;
    for (int j = 0; j < 3; ++j) J[4][1 + j] = 0.5 * s.Sc2c[j];
    J[4][4] = -0.25 * s.Sc2q;
}

// BGK sums by axis factorisation: e = exp(z0) prod_d exp(z_d c_d - z4 c_d^2 / 2).
__device__ void sums_bgk(const NewtonArgs &A, const double U[3], double st, const double z[5], Sums &s) {
    double m[3][5];
    for (int d = 0; d < 3; ++d) {
        double a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0;
        const int nv = A.vg.nv[d];
        for (int i = 0; i < nv; ++i) {
            double c = (gridu(A.vg, d, i) - U[d]) / st;
            double w = A.wax[64 * d + i] / st;
            double ev = w * exp(z[1 + d] * c - 0.5 * z[4] * c * c);
            double t = ev;
            a0 += t; t *= c;
            a1 += t; t *= c;
            a2 += t; t *= c;
            a3 += t; t *= c;
            a4 += t;
        }
        m[d][0] = a0; m[d][1] = a1; m[d][2] = a2; m[d][3] = a3; m[d][4] = a4;
    }
    double K = exp(z[0]) * m[0][0] * m[1][0] * m[2][0];
    double Pn[3][5];
    for (int d = 0; d < 3; ++d)
        for (int a = 0; a < 5; ++a) Pn[d][a] = m[d][a] / m[d][0];
    s.S0 = K;
    for (int i = 0; i < 3; ++i) s.Sc[i] = K * Pn[i][1];
    s.Scc[0] = K * Pn[0][2]; s.Scc[1] = K * Pn[1][2]; s.Scc[2] = K * Pn[2][2];
    s.Scc[3] = K * Pn[0][1] * Pn[1][1];
    s.Scc[4] = K * Pn[0][1] * Pn[2][1];
    s.Scc[5] = K * Pn[1][1] * Pn[2][1];
    s.Sq = s.Scc[0] + s.Scc[1] + s.Scc[2];
    for (int i = 0; i < 3; ++i) {
        double t = 0;
        for (int mm = 0; mm < 3; ++mm) t += (mm == i) ? Pn[i][3] : Pn[i][1] * Pn[mm][2];
        s.Scq[i] = K * t;
        s.Sc2c[i] = K * t;
    }
    double t4 = 0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) t4 += (a == b) ? Pn[a][4] : Pn[a][2] * Pn[b][2];
    s.Sc2q = K * t4;
}

__device__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ES sums over all velocity nodes: lane-strided, butterfly reduced.
__device__ void sums_es(const NewtonArgs &A, int lane, const double U[3], double st, double wscale,
                        const double Am[3][3], const double z[5], Sums &s) {
    double acc[18];
#pragma unroll
    for (int a = 0; a < 18; ++a) acc[a] = 0.0;
    const VGrid &vg = A.vg;
    for (int k = lane; k < vg.nu; k += 64) {
        int i = k % vg.nv[0], j = (k / vg.nv[0]) % vg.nv[1], l = k / (vg.nv[0] * vg.nv[1]);
        double c0 = (gridu(vg, 0, i) - U[0]) / st;
        double c1 = (gridu(vg, 1, j) - U[1]) / st;
        double c2 = (gridu(vg, 2, l) - U[2]) / st;
        double q = Am[0][0] * c0 * c0 + Am[1][1] * c1 * c1 + Am[2][2] * c2 * c2 +
                   2.0 * (Am[0][1] * c0 * c1 + Am[0][2] * c0 * c2 + Am[1][2] * c1 * c2);
        double w = A.wax[i] * A.wax[64 + j] * A.wax[128 + l] * wscale;
        double ev = w * exp(z[0] + z[1] * c0 + z[2] * c1 + z[3] * c2 - 0.5 * z[4] * q);
        double cc = c0 * c0 + c1 * c1 + c2 * c2;
        double eq_ = ev * q, ec = ev * cc;
        acc[0] += ev;
        acc[1] += ev * c0; acc[2] += ev * c1; acc[3] += ev * c2;
        acc[4] += ev * c0 * c0; acc[5] += ev * c1 * c1; acc[6] += ev * c2 * c2;
        acc[7] += ev * c0 * c1; acc[8] += ev * c0 * c2; acc[9] += ev * c1 * c2;
        acc[10] += eq_;
        acc[11] += eq_ * c0; acc[12] += eq_ * c1; acc[13] += eq_ * c2;
        acc[14] += ec * c0; acc[15] += ec * c1; acc[16] += ec * c2;
        acc[17] += ec * q;
    }
    s.S0 = wave_sum(acc[0]);
    for (int d = 0; d < 3; ++d) s.Sc[d] = wave_sum(acc[1 + d]);
    for (int a = 0; a < 6; ++a) s.Scc[a] = wave_sum(acc[4 + a]);
    s.Sq = wave_sum(acc[10]);
    for (int d = 0; d < 3; ++d) s.Scq[d] = wave_sum(acc[11 + d]);
    for (int d = 0; d < 3; ++d) s.Sc2c[d] = wave_sum(acc[14 + d]);
    s.Sc2q = wave_sum(acc[17]);
}

// Closed-form eigenvalues of a symmetric 3x3 matrix; returns the smallest.
__device__ double sym3_min_eig(const double T[3][3]) {
    double p1 = T[0][1] * T[0][1] + T[0][2] * T[0][2] + T[1][2] * T[1][2];
    double q = (T[0][0] + T[1][1] + T[2][2]) / 3.0;
    if (p1 == 0.0) return fmin(T[0][0], fmin(T[1][1], T[2][2]));
    double p2 = (T[0][0] - q) * (T[0][0] - q) + (T[1][1] - q) * (T[1][1] - q) + (T[2][2] - q) * (T[2][2] - q) + 2.0 * p1;
    double p = sqrt(p2 / 6.0);
    double B[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) B[i][j] = (T[i][j] - (i == j ? q : 0.0)) / p;
    double detB = B[0][0] * (B[1][1] * B[2][2] - B[1][2] * B[2][1]) - B[0][1] * (B[1][0] * B[2][2] - B[1][2] * B[2][0]) +
                  B[0][2] * (B[1][0] * B[2][1] - B[1][1] * B[2][0]);
    double r = fmin(1.0, fmax(-1.0, 0.5 * detB));
    double phi = acos(r) / 3.0;
    return q + 2.0 * p * cos(phi + kTwoPi / 3.0);
}

__device__ double det3(const double M[3][3]) {
    return M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
           M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
}

__device__ void inv3(const double M[3][3], double R[3][3]) {
    double d = det3(M);
    R[0][0] = (M[1][1] * M[2][2] - M[1][2] * M[2][1]) / d;
    R[0][1] = (M[0][2] * M[2][1] - M[0][1] * M[2][2]) / d;
    R[0][2] = (M[0][1] * M[1][2] - M[0][2] * M[1][1]) / d;
    R[1][0] = (M[1][2] * M[2][0] - M[1][0] * M[2][2]) / d;
    R[1][1] = (M[0][0] * M[2][2] - M[0][2] * M[2][0]) / d;
    R[1][2] = (M[0][2] * M[1][0] - M[0][0] * M[1][2]) / d;
    R[2][0] = (M[1][0] * M[2][1] - M[1][1] * M[2][0]) / d;
    R[2][1] = (M[0][1] * M[2][0] - M[0][0] * M[2][1]) / d;
    R[2][2] = (M[0][0] * M[1][1] - M[0][1] * M[1][0]) / d;
}

// Equilibrium record and primitive output from the converged parameters.
__device__ void write_point(const NewtonArgs &A, int64_t pt, double rho, const double U[3], double th,
                            const double Am[3][3], const double z[5], double inv_tau, double res) {
    double Ai[3][3];
    inv3(Am, Ai);
    double m[3], mAm = 0;
    for (int i = 0; i < 3; ++i) m[i] = (Ai[i][0] * z[1] + Ai[i][1] * z[2] + Ai[i][2] * z[3]) / z[4];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) mAm += m[i] * Am[i][j] * m[j];
    double st = sqrt(th);
    double *eq = A.eq + pt * kEqW;
    eq[EQ_C0] = log(rho) - 1.5 * log(th) + z[0] + 0.5 * z[4] * mAm;
    for (int d = 0; d < 3; ++d) eq[EQ_V + d] = U[d] + st * m[d];
    double sc = z[4] / th;
    eq[EQ_B] = sc * Am[0][0]; eq[EQ_B + 1] = sc * Am[1][1]; eq[EQ_B + 2] = sc * Am[2][2];
    eq[EQ_B + 3] = sc * Am[0][1]; eq[EQ_B + 4] = sc * Am[0][2]; eq[EQ_B + 5] = sc * Am[1][2];
    eq[EQ_INVTAU] = inv_tau;
    eq[EQ_RES] = res;
    double *pp = A.prim + pt * 5;
    pp[0] = rho * exp(z[0] + 0.5 * z[4] * mAm) * pow(kTwoPi / z[4], 1.5) / sqrt(det3(Am));
    for (int d = 0; d < 3; ++d) pp[1 + d] = eq[EQ_V + d];
    pp[4] = th / z[4];
    for (int a = 0; a < 5; ++a) A.z[pt * 5 + a] = z[a];
}

__device__ void write_nonreal(const NewtonArgs &A, int64_t pt) {
    double *eq = A.eq + pt * kEqW;
    eq[EQ_C0] = -INFINITY;
    for (int a = 1; a < kEqW; ++a) eq[a] = 0.0;
    for (int a = 0; a < 5; ++a) { A.prim[pt * 5 + a] = 0.0; A.z[pt * 5 + a] = 0.0; }
}

// Learned initial guess: MLP on (ln rho, U/u_max, ln theta, u_max/10, n_v/32) -> dz.
__device__ bool mlp_guess(const NewtonArgs &A, double rho, const double U[3], double th, double z[5]);

// Newton iteration shared by both kernels.  Sum evaluation is a functor.
template <typename SumsFn>
__device__ int newton_solve(const NewtonArgs &A, SumsFn sums, const double zc[5], double z[5], double &res,
                            int &iters) {
    double r[5], J[5][5];
    Sums s;
    sums(z, s);
    assemble(s, r, J);
    int conv = 0, it;
    for (it = 0; it < A.max_iter; ++it) {
        double rn = norm2_5(r), ri = normi_5(r);
        double rhs[5] = {-r[0], -r[1], -r[2], -r[3], -r[4]}, dz[5];
        bool ok = solve5(J, rhs, dz);
        if (ok && ri <= A.tol) {
            // converged: one extra full step makes the result path independent
            for (int a = 0; a < 5; ++a) z[a] += dz[a];
            res = ri;
            conv = 1;
            ++it;
            break;
        }
        if (!ok) break;
        double alpha = 1.0, zt[5], rt[5], Jt[5][5];
        bool acc = false;
        for (int hh = 0; hh < 40; ++hh) {
            for (int a = 0; a < 5; ++a) zt[a] = z[a] + alpha * dz[a];
            if (zt[4] > 0.0) {
                Sums st;
                sums(zt, st);
                assemble(st, rt, Jt);
                if (norm2_5(rt) < (1.0 - 1e-4 * alpha) * rn) { acc = true; break; }
            }
            alpha *= 0.5;
        }
        if (!acc) {
            // stagnation at the rounding floor of the FP64 sums
            if (ri <= 100.0 * A.tol) { res = ri; conv = 1; ++it; }
            break;
        }
        for (int a = 0; a < 5; ++a) {
            z[a] = zt[a];
            r[a] = rt[a];
            for (int b = 0; b < 5; ++b) J[a][b] = Jt[a][b];
        }
    }
    iters = it;
    if (!conv) {
        res = normi_5(r);
        for (int a = 0; a < 5; ++a) z[a] = zc[a];
    }
    return conv;
}

__device__ void record_stats(const NewtonArgs &A, int iters, int status, double res) {
    atomicAdd(&A.stats[iters < kHist ? iters : kHist - 1], 1ull);
    if (status == FR_DVM_NEWTON_FALLBACK) atomicAdd(&A.stats[kHist], 1ull);
    if (status == FR_DVM_NEWTON_ESGUARD) atomicAdd(&A.stats[kHist + 1], 1ull);
    if (res >= 0.0 && isfinite(res)) atomicMax(A.maxres, (unsigned long long)__double_as_longlong(res));
}

__device__ bool initial_guess(const NewtonArgs &A, int64_t pt, double rho, const double U[3], double th,
                              const double zc[5], double z[5]) {
    for (int a = 0; a < 5; ++a) z[a] = zc[a];
    if (A.guess == FR_DVM_GUESS_WARM) {
        double zw[5];
        bool ok = true;
        for (int a = 0; a < 5; ++a) { zw[a] = A.z[pt * 5 + a]; ok = ok && isfinite(zw[a]); }
        if (ok && zw[4] > 0.0) for (int a = 0; a < 5; ++a) z[a] = zw[a];
    } else if (A.guess == FR_DVM_GUESS_MLP && A.mlp) {
        double zm[5];
        if (mlp_guess(A, rho, U, th, zm)) for (int a = 0; a < 5; ++a) z[a] = zc[a] + zm[a];
    }
    return true;
}

__global__ __launch_bounds__(256) void k_newton_bgk(const NewtonArgs A) {
    const int64_t pt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pt >= A.npts) return;
    const double *Q = A.Q + pt * A.nmom;
    const double rho = Q[0];
    double U[3] = {Q[1] / rho, Q[2] / rho, Q[3] / rho};
    const double th = (2.0 / 3.0) * (Q[4] / rho - 0.5 * (U[0] * U[0] + U[1] * U[1] + U[2] * U[2]));
    if (!(rho > 0.0) || !(th > 0.0) || !isfinite(rho) || !isfinite(th)) {
        write_nonreal(A, pt);
        record_stats(A, 0, FR_DVM_NEWTON_NONREAL, -1.0);
        return;
    }
    const double inv_tau = rho * th / viscosity(A, th);
    const double st = sqrt(th);
    const double zc[5] = {-1.5 * log(kTwoPi), 0.0, 0.0, 0.0, 1.0};
    double z[5];
    initial_guess(A, pt, rho, U, th, zc, z);
    auto fn = [&](const double zz[5], Sums &s) { sums_bgk(A, U, st, zz, s); };
    double res;
    int iters;
    int conv = newton_solve(A, fn, zc, z, res, iters);
    const double Am[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    write_point(A, pt, rho, U, th, Am, z, inv_tau, res);
    record_stats(A, iters, conv ? FR_DVM_NEWTON_OK : FR_DVM_NEWTON_FALLBACK, res);
}

__global__ __launch_bounds__(256) void k_newton_es(const NewtonArgs A) {
    const int lane = threadIdx.x & 63;
    const int64_t pt = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (pt >= A.npts) return;  // whole waves exit together
    const double *Q = A.Q + pt * A.nmom;
    const double rho = Q[0];
    double U[3] = {Q[1] / rho, Q[2] / rho, Q[3] / rho};
    // raw second moments -> pressure tensor Pi = M2 - rho U U^T
    double Pi[6] = {Q[4] - rho * U[0] * U[0], Q[5] - rho * U[1] * U[1], Q[6] - rho * U[2] * U[2],
                    Q[7] - rho * U[0] * U[1], Q[8] - rho * U[0] * U[2], Q[9] - rho * U[1] * U[2]};
    const double th = (Pi[0] + Pi[1] + Pi[2]) / (3.0 * rho);
    if (!(rho > 0.0) || !(th > 0.0) || !isfinite(rho) || !isfinite(th)) {
        if (lane == 0) {
            write_nonreal(A, pt);
            record_stats(A, 0, FR_DVM_NEWTON_NONREAL, -1.0);
        }
        return;
    }
    const double Pr = A.Pr;
    const double inv_tau = Pr * rho * th / viscosity(A, th);
    const double st = sqrt(th);
    double Am[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    int status = FR_DVM_NEWTON_OK;
    {
        double a1 = th / Pr, a2 = (1.0 - 1.0 / Pr) / rho;
        double T[3][3] = {{a1 + a2 * Pi[0], a2 * Pi[3], a2 * Pi[4]},
                          {a2 * Pi[3], a1 + a2 * Pi[1], a2 * Pi[5]},
                          {a2 * Pi[4], a2 * Pi[5], a1 + a2 * Pi[2]}};
        if (sym3_min_eig(T) <= 1e-8 * th) {
            status = FR_DVM_NEWTON_ESGUARD;
        } else {
            double Ti[3][3];
            inv3(T, Ti);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) Am[i][j] = th * Ti[i][j];
        }
    }
    const double zc[5] = {-1.5 * log(kTwoPi) + 0.5 * log(det3(Am)), 0.0, 0.0, 0.0, 1.0};
    double z[5];
    initial_guess(A, pt, rho, U, th, zc, z);
    const double wscale = 1.0 / (th * st);
    auto fn = [&](const double zz[5], Sums &s) { sums_es(A, lane, U, st, wscale, Am, zz, s); };
    double res;
    int iters;
    int conv = newton_solve(A, fn, zc, z, res, iters);
    if (lane == 0) {
        write_point(A, pt, rho, U, th, Am, z, inv_tau, res);
        record_stats(A, iters, conv ? status : FR_DVM_NEWTON_FALLBACK, res);
    }
}

// MLP: 7 -> H -> H -> H -> 5, SiLU, FP32 weights packed layer by layer as
// [W (out x in, row major), b (out)], plus 5 output scales and 5 offsets.
__device__ bool mlp_guess(const NewtonArgs &A, double rho, const double U[3], double th, double z[5]) {
    const int H = A.mlp_hidden;
    if (H <= 0 || H > 64) return false;
    double umax = 0;
    for (int d = 0; d < 3; ++d) umax = fmax(umax, fmax(fabs(A.vg.umin[d]), fabs(A.vg.umin[d] + (A.vg.nv[d] - 1) * A.vg.du[d])));
    float x[64], y[64];
    x[0] = (float)log(rho);
    for (int d = 0; d < 3; ++d) x[1 + d] = (float)(U[d] / umax);
    x[4] = (float)log(th);
    x[5] = (float)(umax / 10.0);
    x[6] = (float)(A.vg.nv[0] / 32.0);
    const float *w = A.mlp;
    int nin = 7;
    for (int layer = 0; layer < 4; ++layer) {
        int nout = layer == 3 ? 5 : H;
        const float *W = w, *b = w + nout * nin;
        for (int o = 0; o < nout; ++o) {
            float s = b[o];
            for (int i = 0; i < nin; ++i) s += W[o * nin + i] * x[i];
            y[o] = layer == 3 ? s : s / (1.0f + __expf(-s));
        }
        w = b + nout;
        for (int o = 0; o < nout; ++o) x[o] = y[o];
        nin = nout;
    }
    for (int a = 0; a < 5; ++a) {
        z[a] = (double)(x[a] * w[a] + w[5 + a]);
        if (!isfinite(z[a])) return false;
    }
    return true;
}

__global__ void k_collide(const VGrid vg, const double *__restrict__ eqs, const void *fv, void *Sv, int accumulate,
                          int fp64) {
    const int64_t pt = blockIdx.x;
    const double *eqp = eqs + pt * kEqW;
    double eq[kEqW];
    for (int a = 0; a < kEqW; ++a) eq[a] = eqp[a];
    for (int k = threadIdx.x; k < vg.nu; k += blockDim.x) {
        int i = k % vg.nv[0], j = (k / vg.nv[0]) % vg.nv[1], l = k / (vg.nv[0] * vg.nv[1]);
        double u[3] = {gridu(vg, 0, i), gridu(vg, 1, j), gridu(vg, 2, l)};
        int64_t idx = pt * vg.nu + k;
        if (fp64) {
            double c0 = u[0] - eq[EQ_V], c1 = u[1] - eq[EQ_V + 1], c2 = u[2] - eq[EQ_V + 2];
            double q = eq[EQ_B] * c0 * c0 + eq[EQ_B + 1] * c1 * c1 + eq[EQ_B + 2] * c2 * c2 +
                       2.0 * (eq[EQ_B + 3] * c0 * c1 + eq[EQ_B + 4] * c0 * c2 + eq[EQ_B + 5] * c1 * c2);
            double g = exp(eq[EQ_C0] - 0.5 * q);
            double f = ((const double *)fv)[idx];
            double S = (g - f) * eq[EQ_INVTAU];
            double *So = (double *)Sv;
            So[idx] = accumulate ? So[idx] + S : S;
        } else {
            float c0 = (float)(u[0] - eq[EQ_V]), c1 = (float)(u[1] - eq[EQ_V + 1]), c2 = (float)(u[2] - eq[EQ_V + 2]);
            float q = (float)eq[EQ_B] * c0 * c0 + (float)eq[EQ_B + 1] * c1 * c1 + (float)eq[EQ_B + 2] * c2 * c2 +
                      2.0f * ((float)eq[EQ_B + 3] * c0 * c1 + (float)eq[EQ_B + 4] * c0 * c2 + (float)eq[EQ_B + 5] * c1 * c2);
            float g = __expf((float)eq[EQ_C0] - 0.5f * q);
            float f = ((const float *)fv)[idx];
            float S = (g - f) * (float)eq[EQ_INVTAU];
            float *So = (float *)Sv;
            So[idx] = accumulate ? So[idx] + S : S;
        }
    }
}

__global__ void k_moments_out(int64_t npts, int nmom, const double *__restrict__ Q, double *__restrict__ out) {
    int64_t pt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pt >= npts) return;
    const double *q = Q + pt * nmom;
    double *o = out + pt * 5;
    o[0] = q[0]; o[1] = q[1]; o[2] = q[2]; o[3] = q[3];
    o[4] = nmom == 5 ? q[4] : 0.5 * (q[4] + q[5] + q[6]);
}

// Domain totals: one workgroup, fixed-order strided sums and tree reduction.
__global__ __launch_bounds__(1024) void k_totals(int64_t npts, int nmom, const double *__restrict__ Q,
                                                 const double *__restrict__ wJ, double *__restrict__ out) {
    __shared__ double red[5][1024];
    double a[5] = {0, 0, 0, 0, 0};
    for (int64_t pt = threadIdx.x; pt < npts; pt += 1024) {
        const double *q = Q + pt * nmom;
        double w = wJ[pt];
        a[0] += w * q[0]; a[1] += w * q[1]; a[2] += w * q[2]; a[3] += w * q[3];
        a[4] += w * (nmom == 5 ? q[4] : 0.5 * (q[4] + q[5] + q[6]));
    }
    for (int c = 0; c < 5; ++c) red[c][threadIdx.x] = a[c];
    __syncthreads();
    for (int o = 512; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o)
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

}  // namespace

int launch_newton(fr_dvm *h, int guess) {
    NewtonArgs A;
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
    A.model = h->prm.model;
    A.Pr = h->prm.prandtl;
    A.mu_ref = h->prm.mu_ref;
    A.theta_ref = h->prm.theta_ref;
    A.omega = h->prm.omega;
    A.theta_s = h->prm.theta_s;
    A.visc_law = h->prm.visc_law;
    A.tol = h->prm.newton_tol;
    A.max_iter = h->prm.newton_max_iter;
    A.guess = (guess == FR_DVM_GUESS_WARM && !h->zvalid) ? FR_DVM_GUESS_COLD : guess;
    A.mlp = h->d_mlp;
    A.mlp_hidden = h->mlp_hidden;
    if (h->prm.model == FR_DVM_ESBGK) {
        hipLaunchKernelGGL(k_newton_es, dim3((unsigned)((A.npts + 3) / 4)), dim3(256), 0, h->stream, A);
    } else {
        hipLaunchKernelGGL(k_newton_bgk, dim3((unsigned)((A.npts + 255) / 256)), dim3(256), 0, h->stream, A);
    }
    h->zvalid = 1;
    return check(h, "newton kernel");
}

int launch_collide(fr_dvm *h, const void *f, void *S, int accumulate) {
    hipLaunchKernelGGL(k_collide, dim3((unsigned)(h->ne * h->ns)), dim3(256), 0, h->stream, h->vg, h->d_eq, f, S,
                       accumulate, h->prm.precision == FR_DVM_FP64 ? 1 : 0);
    return check(h, "collide kernel");
}

int launch_prim_out(fr_dvm *h, double *Qp) {
    if (hipMemcpyAsync(Qp, h->d_prim, sizeof(double) * 5 * h->ne * h->ns, hipMemcpyDeviceToDevice, h->stream) !=
        hipSuccess)
        return h->fail(FR_DVM_EHIP, "copy of Q'");
    return FR_DVM_OK;
}

int launch_moments_out(fr_dvm *h, double *Q) {
    int64_t npts = h->ne * h->ns;
    hipLaunchKernelGGL(k_moments_out, dim3((unsigned)((npts + 255) / 256)), dim3(256), 0, h->stream, npts, h->nmom,
                       h->d_Q, Q);
    return check(h, "moments output kernel");
}

int launch_totals(fr_dvm *h, double *host_tot) {
    int64_t npts = h->ne * h->ns;
    hipLaunchKernelGGL(k_totals, dim3(1), dim3(1024), 0, h->stream, npts, h->nmom, h->d_Q, h->d_wq3J, h->d_tot);
    int rc = check(h, "totals kernel");
    if (rc) return rc;
    if (hipMemcpyAsync(host_tot, h->d_tot, 5 * sizeof(double), hipMemcpyDeviceToHost, h->stream) != hipSuccess)
        return h->fail(FR_DVM_EHIP, "totals copy");
    if (hipStreamSynchronize(h->stream) != hipSuccess) return h->fail(FR_DVM_EHIP, "stream synchronise");
    return FR_DVM_OK;
}

}  // namespace frdvm
