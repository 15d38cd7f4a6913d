// Internal declarations of libfrdvm: the handle, kernel argument blocks and
// the launchers implemented in the .hip translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fr_dvm.h"
#include "../../include/fr_dvm_mlp.h"

namespace frdvm {

constexpr int kMaxP = 3;
constexpr int kMaxN = kMaxP + 1;
constexpr int kEqW = 12;   // per-point equilibrium record (see EqRec below)
// per-element reference of the FP32 deviation storage: 10 coefficients of
// its exponent polynomial, then its moments (5 or 10)
constexpr int kRefW = 20;
constexpr int kHist = 64;  // Newton iteration histogram bins

// Per-point equilibrium record written by the Newton kernels and read by the
// collision (fused or stand-alone):
//   g(u) = exp(c0 - 1/2 (u-V)^T B (u-V)),  S = (g - f) * inv_tau
enum EqRec { EQ_C0 = 0, EQ_V = 1, EQ_B = 4 /* xx yy zz xy xz yz */, EQ_INVTAU = 10, EQ_RES = 11 };

// One-dimensional FR operators on Gauss-Legendre points (n = p+1 <= 4).
struct Ops1D {
    double D[kMaxN * kMaxN];  // D[i*n+m] = l_m'(xi_i)
    double lam[2][kMaxN];     // lam[side][m] = l_m(-1 | +1)
    double corr[2][kMaxN];    // corr[side][i]: correction derivative at xi_i for a unit jump on face side
    double wq[kMaxN];         // Gauss weights
    double xi[kMaxN];
};

// Velocity grid on the device side: per-axis uniform nodes.
struct VGrid {
    int nv[3];
    int nu;
    double umin[3], du[3];
    int neg_end[3];    // nodes with u_d < 0 are idx < neg_end
    int pos_start[3];  // nodes with u_d > 0 are idx >= pos_start
};

// Compact "outflow half" trace layout for axis-aligned box meshes.  For face
// (d, side) only velocities leaving the element through it are stored:
// side 1: idx_d >= pos_start_d, side 0: idx_d < neg_end_d.
struct TraceLayout {
    int64_t cnt[6];       // velocity entries per face point
    int64_t face_off[6];  // offset of the face block inside the element block
    int64_t elem;         // element block size
};

struct Handle;

// Mixed meshes (fr_dvm_create_mixed): per element type, the reference
// operators of the nodal DG / FR-DG scheme and the elements of that type.
constexpr int kMixGeo = 33;  // per element: dxi/dx (9), unit outward face normals (6x3), |J_face| / |J| (6)
struct MixType {
    int etype = -1, ns = 0, nft = 0, nface = 0;
    std::vector<int32_t> fnode;  // [nft] solution point of each face point (faces in order)
    std::vector<int32_t> ffac;   // [nft] face of each face point
    std::vector<double> D;       // [3][ns][ns] reference derivatives
    std::vector<double> lift;    // [nft][ns] correction of a unit jump at each face point
    std::vector<double> W;       // [ns] integral of each Lagrange function (reference)
    std::vector<int32_t> elems;  // elements of this type
    double *d_D = nullptr, *d_lift = nullptr;
    float *d_Df = nullptr, *d_liftf = nullptr;
    int32_t *d_elems = nullptr, *d_fnode = nullptr, *d_ffac = nullptr;
};
struct Mixed {
    int64_t ne = 0, npts = 0, nfp = 0;  // elements, solution points, face points (all elements)
    std::vector<int64_t> poff, toff;    // [ne+1] first solution point / face point of each element
    int64_t *d_poff = nullptr, *d_toff = nullptr;
    int64_t *d_tnb = nullptr;           // [nfp] the neighbour's face point at the same position
    double *d_geo = nullptr;            // [ne][kMixGeo]
    float *d_geof = nullptr;
    MixType t[3];
};

}  // namespace frdvm

struct fr_dvm {
    std::string err;
    hipStream_t stream = nullptr;
    int device = 0;
    // second stream for the Newton solves overlapped with the stage launches,
    // and the events that order the two (stage half done, Newton half done)
    hipStream_t aux = nullptr;
    hipEvent_t ev_stage[2] = {nullptr, nullptr}, ev_newton[2] = {nullptr, nullptr};

    // discretisation
    int p = 0, n = 0, ns = 0, nfp = 0;
    int nodes = 0;  // solution points: 0 Gauss-Legendre, 1 Gauss-Lobatto
    double delta = 0;  // internal degrees of freedom of the gas
    int ncomp = 1;     // 1: f; 2: the reduced pair (F, G), per point F then G (nu values each)
    // mixed meshes: every solution point is an "element" of one point for the
    // point-wise machinery (ne = points, ns = 1); the element structure is here
    frdvm::Mixed *mx = nullptr;
    int64_t ne = 0;
    frdvm::VGrid vg{};
    std::vector<double> wax[3];  // 1-D trapezoid weights per axis
    frdvm::Ops1D ops{};
    bool axis_mode = false;
    frdvm::TraceLayout tl{};
    double hmin = 0;

    // copy of the caller's mesh of a box handle, kept so that enabling the
    // positivity limiter can move the handle to the general-mesh path
    struct MeshCopy {
        int32_t n_elem = 0, n_nodes = 0, geom_order = 0;
        std::vector<double> nodes;
        std::vector<int32_t> elem_nodes, nbr_elem;
        std::vector<int8_t> nbr_face, nbr_orient, bc;
    } mesh_copy;

    // host geometry (for totals / dt)
    std::vector<double> h_gfac;  // [ne][3]  2/h_d for axis boxes
    std::vector<double> h_detJ;  // [ne][ns]

    // device: geometry and tables
    double *d_gfac = nullptr;    // [ne][3]
    // general (curved / re-oriented / bounded) meshes, axis_mode == false
    double *d_S = nullptr;       // [ne][ns][3][3] S[d][c] = (|J| J^-1)_dc, rows a^d = |J| grad xi_d
    double *d_ijac = nullptr;    // [ne][ns] 1/|J|
    double *d_nf = nullptr;      // [ne][6][nfp][3] outward area-scaled normal at the flux points
    float *d_Sf = nullptr, *d_ijacf = nullptr, *d_nff = nullptr;  // FP32 copies
    int32_t *d_conn = nullptr;   // [ne][6][4] neighbour, its face, orientation code, bc tag
    int32_t *d_wall = nullptr;   // [nwall] e*6+face of every diffuse-wall face
    int64_t nwall = 0;
    double *d_rw = nullptr;      // [ne*6][nfp] wall-Maxwellian density of the current stage
    double *d_mw = nullptr;      // [nu] unit-density wall Maxwellian at theta_wall
    double *d_finf = nullptr;    // [ncomp * nu] farfield Maxwellian (and its G)
    double *d_gfp = nullptr;     // [ne*ns] delta theta / 2 of each point (the pair's G equilibrium factor)
    int32_t *d_nbr = nullptr;    // [ne][6]
    double *d_wq3J = nullptr;    // [ne*ns] Gauss weight x |J| per solution point
    double *d_wx3 = nullptr;     // [nv_x][3] moment weights along x: w, w u_x, w u_x^2
    double *d_wrow = nullptr;    // [nv_y nv_z][6] per (y,z) row: W, W u_y, W u_z, W u_y^2, W u_z^2, W u_y u_z
    double *d_wax = nullptr;     // [3][64] 1-D weights

    // parameters
    fr_dvm_params prm{};
    bool have_params = false;
    int nmom = 5;                // 5 (BGK) or 10 (ES: rho, rho U, raw second moments)
    bool es_direct = false;      // ES Newton: force the direct per-node sums (env FRDVM_ES_DIRECT=1)

    // work buffers
    void *d_reg = nullptr;       // second RK register [ne*ns*nu]
    void *d_tr[2] = {nullptr, nullptr};
    int cur_tr = 0;
    double *d_Q = nullptr;       // [ne*ns][nmom]
    double *d_eq = nullptr;      // [ne*ns][kEqW]
    // [ne][kRefW] element references (FP32 deviation storage): three sets,
    // those of the value read by a stage, of its result, and (SSP) of the
    // step's initial value
    double *d_ref[3] = {nullptr, nullptr, nullptr};
    int cur_ref = 0, prev_ref = 0, u0_ref = 0;
    double *d_z = nullptr;       // [ne*ns][5] Newton solution (warm start)
    double *d_prim = nullptr;    // [ne*ns][5] primitive state of g(Q')
    int zvalid = 0;
    uint32_t stage_count = 0;   // RK stages since fr_dvm_set_params (seeds of the stochastic rounding)
    bool newton_done = false;    // a solve has filled the per-point outcome arrays
    int32_t *d_pt_iters = nullptr;   // [ne*ns] per-point Newton outcome of the last solve
    int32_t *d_pt_evals = nullptr;
    int32_t *d_pt_status = nullptr;
    double *d_pt_resid = nullptr;
    int64_t *d_stats = nullptr;  // [kHist + 4]: histogram, fallback, ES guard, evaluations
    double *d_maxres = nullptr;  // [1] (as ordered bits)
    double *d_tot = nullptr;     // [5]
    float *d_mlp = nullptr;      // learned-guess network weights
    size_t mlp_n = 0;
    int mlp_hidden = 0;
    float *d_mlp_x = nullptr;    // feature batch
    float *d_mlp_work = nullptr; // forward workspace
    float *d_mlp_dz = nullptr;   // [npts][5] predicted Newton corrections
    size_t mlp_x_n = 0, mlp_work_n = 0, dz_n = 0;
    size_t owned_bytes = 0;

    // HIP-event kernel timing (fr_dvm_profile)
    bool prof = false;
    struct ProfRec { int kind; hipEvent_t a, b; };
    std::vector<ProfRec> prof_recs;
    double prof_ms[FR_DVM_PROF_KINDS] = {0, 0, 0, 0};
    int64_t prof_n[FR_DVM_PROF_KINDS] = {0, 0, 0, 0};

    int fail(int code, const std::string &m) { err = m; return code; }
};

namespace frdvm {
// Brackets a launch with events when profiling is on.
struct ProfScope {
    fr_dvm *h;
    int kind;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    // s: the stream the timed launches go to (nullptr: the handle's stream)
    ProfScope(fr_dvm *h_, int k, hipStream_t s_ = nullptr) : h(h_), kind(k), s(s_ ? s_ : h_->stream) {
        if (h->prof && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
            (void)hipEventRecord(a, s);
    }
    ~ProfScope() {
        if (a && b) {
            (void)hipEventRecord(b, s);
            h->prof_recs.push_back({kind, a, b});
        }
    }
};
}  // namespace frdvm

namespace frdvm {

// ---- launchers (frdvm_fr.hip) ----
// mode: 0 = prime (traces + moments of f), 1 = stage (RK update of f into
// fout, traces + moments of the result), 2 = residual only (R into fout).
struct StageArgs {
    const void *f;      // current stage value
    const void *fn;     // f^n (SSP) or dF (LSRK), may be null at stage 1
    void *fout;         // output register
    void *dF;           // LSRK dF register (in/out)
    const void *tr_in;  // neighbour traces of f
    void *tr_out;       // own outflow traces of the result
    double *Q;          // moments of the result [ne*ns][nmom]
    const double *eq;   // equilibrium records [ne*ns][kEqW]
    double dt, alpha, beta;  // SSP: fout = alpha fn + beta (f + dt L)
    double lsA, lsB;         // LSRK: dF = lsA dF + dt L; fout = f + lsB dF
    int scheme;              // 0 SSP, 1 LSRK
    int keep_dF;             // LSRK: store dF (not after the last stage of a step, where it is dead)
    int collide;             // include the collision source
    int positivity;          // limit the stage result to f >= 0 (general-mesh kernel)
    // FP32 deviation storage (FR_DVM_FP32_DEV): the stage value and the
    // inflow traces are read as deviations from the element references of
    // the previous stage's records (in_dev; else plain, made relative here)
    // and the result written as the deviation from the element's reference
    // of this stage's records (out_dev; else plain); SSP: the step's initial
    // value fn relative to ref_u0 (fn_dev; else plain)
    const double *ref_prev, *ref_cur, *ref_u0;  // [ne][kRefW]
    int in_dev, out_dev, fn_dev;
    uint32_t seed;           // random bits of the stage's stochastic rounding of FP32 state values
    int64_t e0, ecount;      // element range [e0, e0 + ecount); ecount 0: all elements
};
int launch_fr_axis(fr_dvm *h, int mode, const StageArgs &a, int do_traces, int do_moments);
// element references of the current equilibrium records into ref [ne][kRefW]
int launch_elem_ref(fr_dvm *h, double *ref);
// ---- mixed meshes (frdvm_gen.hip): same modes and arguments ----
int launch_fr_mixed(fr_dvm *h, int mode, const StageArgs &a, int do_traces, int do_moments);
// ---- general meshes (frdvm_gen.hip): same modes and arguments ----
int launch_fr_gen(fr_dvm *h, int mode, const StageArgs &a, int do_traces, int do_moments);
// boundary tables of the current parameters (wall and farfield Maxwellians)
int gen_boundary_tables(fr_dvm *h);
inline int launch_fr(fr_dvm *h, int mode, const StageArgs &a, int do_traces, int do_moments) {
    if (h->mx) return launch_fr_mixed(h, mode, a, do_traces, do_moments);
    return h->axis_mode ? launch_fr_axis(h, mode, a, do_traces, do_moments)
                        : launch_fr_gen(h, mode, a, do_traces, do_moments);
}

// ---- host set-up shared by the mesh kinds (frdvm_setup.cpp) ----
void gauss_legendre_rule(int n, double *x, double *w);
void gauss_lobatto_rule(int n, double *x, double *w);
int setup_vgrid(fr_dvm *h, const fr_dvm_vgrid *grid);
int finish_create(fr_dvm *h, const std::vector<double> &wq3J);
// ---- mixed meshes (frdvm_mixed.cpp) ----
void free_mixed(fr_dvm *h);

// ---- launchers (frdvm_newton.hip) ----
int launch_newton(fr_dvm *h, int guess);
// Newton over the points [p0, p0 + np) on stream s (warm or cold start only;
// newton_part_ok tells whether the handle's start allows it).
int newton_part_ok(fr_dvm *h, int guess);
int launch_newton_part(fr_dvm *h, int guess, int64_t p0, int64_t np, hipStream_t s);
int launch_newton_points(fr_dvm *h, const double *Q, int64_t n, int guess, double *z, int32_t *iters, int32_t *evals,
                         int32_t *status, double *resid);
int launch_collide(fr_dvm *h, const void *f, void *S, int accumulate);
int launch_prim_out(fr_dvm *h, double *Qp);
int launch_moments_out(fr_dvm *h, double *Q);
int launch_totals(fr_dvm *h, double *host_tot);
int launch_kn_gll(fr_dvm *h, double *kn);

}  // namespace frdvm
