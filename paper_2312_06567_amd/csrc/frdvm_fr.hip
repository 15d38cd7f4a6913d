// Fused FR residual + collision + Runge-Kutta stage kernel for axis-aligned
// hexahedral box meshes (gfx950).
//
// Paper, Section "Numerical method": every velocity node u0 is advected by
// its own FR scheme (eq. transport): interpolate the element polynomial to
// the flux nodes, take the upwind common flux F^I = u_n f- (u_n > 0) or
// u_n f+ (otherwise), and add to the flux divergence the correction
// [F^I - u_n f-] times the divergence of the DG-recovering correction
// function.  The collision source (g(Q') - f)/tau follows Section
// "Governing equations"; Q' comes from the Newton kernels.
//
// Work decomposition: one workgroup (4 wave64) per element; each lane owns
// one velocity node and holds the element's (p+1)^3 solution values in
// registers.  On a tensor-product Gauss element every operator factorises
// along lines, so the divergence is 3 (p+1)^4 FMAs and each face trace or
// correction touches only the line through its flux node: the kernel is HBM
// bound and uses plain VALU FMAs (no MFMA: the sum-factorised contraction has
// K = p+1 <= 4).
//
// Traces: each element stores, for the velocities leaving it through a face,
// its trace on that face ("outflow half", compact layout) into the trace
// buffer of the next stage; the downwind neighbour reads exactly those
// entries as its exterior state.  Two trace buffers alternate between stages.
//
// Moments of the produced stage value are reduced inside the kernel: each
// wave transposes its 64-velocity x NS-point tile through LDS so that a lane
// owns one solution point, and accumulates sum_k w_k psi_k f_k in FP64 with
// wave-uniform (scalar) weights.  The sum order is fixed: results are
// bitwise reproducible run to run.
#include <hip/hip_runtime.h>

#include "frdvm_common.h"

namespace frdvm {

namespace {

constexpr int MODE_PRIME = 0, MODE_STAGE = 1, MODE_RESID = 2;

struct FrArgs {
    Ops1D ops;
    VGrid vg;
    TraceLayout tl;
    int64_t ne;
    int nu;
    const double *gfac;   // [ne][3]
    const int32_t *nbr;   // [ne][6]
    const double *wpsi;   // [nu_pad][NMOM]
    StageArgs sa;
    int do_traces, do_moments;
};

__device__ __forceinline__ int compact_index(const VGrid &vg, int d, int side, const int iv[3]) {
    int idx[3] = {iv[0], iv[1], iv[2]};
    int ext[3] = {vg.nv[0], vg.nv[1], vg.nv[2]};
    if (side) {
        idx[d] -= vg.pos_start[d];
        ext[d] = vg.nv[d] - vg.pos_start[d];
    } else {
        ext[d] = vg.neg_end[d];
    }
    return idx[0] + ext[0] * (idx[1] + ext[1] * idx[2]);
}

template <int N>
__device__ __forceinline__ constexpr int line_pt(int d, int fp, int m) {
    // solution index of the m-th point along axis d through face point fp = a + N b
    return d == 0 ? m + N * fp : (d == 1 ? (fp % N) + N * (m + N * (fp / N)) : fp + N * N * m);
}

template <typename Real>
__device__ __forceinline__ Real eval_g(const double *eq, const double u[3]);

template <>
__device__ __forceinline__ double eval_g<double>(const double *eq, const double u[3]) {
    double c0 = u[0] - eq[EQ_V], c1 = u[1] - eq[EQ_V + 1], c2 = u[2] - eq[EQ_V + 2];
    double q = eq[EQ_B] * c0 * c0 + eq[EQ_B + 1] * c1 * c1 + eq[EQ_B + 2] * c2 * c2 +
               2.0 * (eq[EQ_B + 3] * c0 * c1 + eq[EQ_B + 4] * c0 * c2 + eq[EQ_B + 5] * c1 * c2);
    return exp(eq[EQ_C0] - 0.5 * q);
}

template <>
__device__ __forceinline__ float eval_g<float>(const double *eq, const double u[3]) {
    // differences of O(u_max) numbers in FP64, the quadratic form and exp in FP32
    float c0 = (float)(u[0] - eq[EQ_V]), c1 = (float)(u[1] - eq[EQ_V + 1]), c2 = (float)(u[2] - eq[EQ_V + 2]);
    float q = (float)eq[EQ_B] * c0 * c0 + (float)eq[EQ_B + 1] * c1 * c1 + (float)eq[EQ_B + 2] * c2 * c2 +
              2.0f * ((float)eq[EQ_B + 3] * c0 * c1 + (float)eq[EQ_B + 4] * c0 * c2 + (float)eq[EQ_B + 5] * c1 * c2);
    return __expf((float)eq[EQ_C0] - 0.5f * q);
}

template <typename Real, int P, int NMOM, int MODE>
__global__ __launch_bounds__(kBlock) void k_fr_axis(const FrArgs A) {
    constexpr int N = P + 1, NS = N * N * N, NFP = N * N;
    constexpr int TILE_LD = 33;  // padded row of the transpose tile
    // LDS: equilibrium records, then a union of the transpose tiles and the
    // cross-wave reduction buffer
    __shared__ double s_eq[(MODE == MODE_STAGE) ? NS * kEqW : 1];
    constexpr size_t TILE_BYTES = sizeof(Real) * 4 * NS * TILE_LD;
    constexpr size_t RED_BYTES = sizeof(double) * 4 * NS * NMOM;
    __shared__ __attribute__((aligned(16))) unsigned char s_raw[TILE_BYTES > RED_BYTES ? TILE_BYTES : RED_BYTES];
    Real(*tile)[NS][TILE_LD] = reinterpret_cast<Real(*)[NS][TILE_LD]>(s_raw);
    double(*red)[NS][NMOM] = reinterpret_cast<double(*)[NS][NMOM]>(s_raw);

    const int64_t e = blockIdx.x;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const VGrid &vg = A.vg;
    const int nu = A.nu;
    const int64_t ebase = e * (int64_t)NS * nu;

    if (MODE == MODE_STAGE && A.sa.collide) {
        for (int i = tid; i < NS * kEqW; i += kBlock) s_eq[i] = A.sa.eq[e * NS * kEqW + i];
    }
    __syncthreads();

    const double gx = A.gfac[3 * e], gy = A.gfac[3 * e + 1], gz = A.gfac[3 * e + 2];
    const double gf[3] = {gx, gy, gz};

    double acc[NMOM];
#pragma unroll
    for (int a = 0; a < NMOM; ++a) acc[a] = 0.0;

    const Real *__restrict__ fin = reinterpret_cast<const Real *>(A.sa.f) + ebase;
    const int nchunk = (nu + kBlock - 1) / kBlock;

    for (int ch = 0; ch < nchunk; ++ch) {
        const int k = ch * kBlock + tid;
        const bool act = k < nu;
        const int kk = act ? k : 0;
        int iv[3];
        iv[0] = kk % vg.nv[0];
        iv[1] = (kk / vg.nv[0]) % vg.nv[1];
        iv[2] = kk / (vg.nv[0] * vg.nv[1]);
        // The sign of each velocity component is taken from the integer
        // split of the grid computed on the host (not from the rounded
        // value), so the compact trace slots of writer and reader always
        // agree; a node classified as zero carries exactly zero flux.
        double u[3];
        int sgn[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            sgn[d] = iv[d] >= vg.pos_start[d] ? 1 : (iv[d] < vg.neg_end[d] ? -1 : 0);
            u[d] = sgn[d] == 0 ? 0.0 : __dadd_rn(vg.umin[d], __dmul_rn((double)iv[d], vg.du[d]));
        }

        Real f[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) f[s] = act ? fin[(int64_t)s * nu + k] : Real(0);

        if (MODE != MODE_PRIME) {
            Real r[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) r[s] = Real(0);
            // flux divergence: sum_d a_d D_d f along every line, a_d = (2/h_d) u_d
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const Real ad = (Real)(gf[d] * u[d]);
#pragma unroll
                for (int fp = 0; fp < NFP; ++fp) {
#pragma unroll
                    for (int i = 0; i < N; ++i) {
                        Real t = Real(0);
#pragma unroll
                        for (int m = 0; m < N; ++m) t += (Real)A.ops.D[i * N + m] * f[line_pt<N>(d, fp, m)];
                        r[line_pt<N>(d, fp, i)] += ad * t;
                    }
                }
            }
            // interface corrections on the inflow face of each axis: the
            // common flux is the neighbour's value, jump = u_n (f+ - f-)
            const Real *__restrict__ trin = reinterpret_cast<const Real *>(A.sa.tr_in);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                if (act && sgn[d] != 0) {
                    const int side_in = sgn[d] > 0 ? 0 : 1;
                    const int nface = 2 * d + (side_in ^ 1);  // neighbour's outflow face
                    const int64_t nb = A.nbr[6 * e + 2 * d + side_in];
                    const int64_t cnt = A.tl.cnt[nface];
                    const int64_t base = nb * A.tl.elem + A.tl.face_off[nface] + compact_index(vg, d, side_in ^ 1, iv);
                    const Real un = (Real)((side_in ? 1.0 : -1.0) * gf[d] * u[d]);
#pragma unroll
                    for (int fp = 0; fp < NFP; ++fp) {
                        const Real fplus = trin[base + fp * cnt];
                        Real fminus = Real(0);
#pragma unroll
                        for (int m = 0; m < N; ++m) fminus += (Real)A.ops.lam[side_in][m] * f[line_pt<N>(d, fp, m)];
                        const Real jmp = un * (fplus - fminus);
#pragma unroll
                        for (int m = 0; m < N; ++m) r[line_pt<N>(d, fp, m)] += (Real)A.ops.corr[side_in][m] * jmp;
                    }
                }
            }
            if (MODE == MODE_RESID) {
                Real *__restrict__ out = reinterpret_cast<Real *>(A.sa.fout) + ebase;
                if (act) {
#pragma unroll
                    for (int s = 0; s < NS; ++s) out[(int64_t)s * nu + k] = -r[s];
                }
                continue;
            }
            // collision source and the Runge-Kutta combination, point by point
            Real *__restrict__ out = reinterpret_cast<Real *>(A.sa.fout) + ebase;
            const Real *__restrict__ fnp = reinterpret_cast<const Real *>(A.sa.fn) + ebase;
            Real *__restrict__ dF = reinterpret_cast<Real *>(A.sa.dF) + ebase;
            const Real dt = (Real)A.sa.dt;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                Real L = -r[s];
                if (A.sa.collide) {
                    const double *eq = &s_eq[s * kEqW];
                    const Real g = eval_g<Real>(eq, u);
                    L += (g - f[s]) * (Real)eq[EQ_INVTAU];
                }
                Real fo;
                if (A.sa.scheme == 0) {
                    fo = (Real)A.sa.beta * (f[s] + dt * L);
                    if (A.sa.alpha != 0.0 && act) fo += (Real)A.sa.alpha * fnp[(int64_t)s * nu + k];
                } else {
                    Real dd = dt * L;
                    if (A.sa.lsA != 0.0 && act) dd += (Real)A.sa.lsA * dF[(int64_t)s * nu + k];
                    if (act) dF[(int64_t)s * nu + k] = dd;
                    fo = f[s] + (Real)A.sa.lsB * dd;
                }
                f[s] = act ? fo : Real(0);
                if (act) out[(int64_t)s * nu + k] = fo;
            }
        }

        // outflow traces of the produced value (the next stage's exterior states)
        if (A.do_traces && act) {
            Real *__restrict__ trout = reinterpret_cast<Real *>(A.sa.tr_out);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                if (sgn[d] != 0) {
                    const int side = sgn[d] > 0 ? 1 : 0;
                    const int face = 2 * d + side;
                    const int64_t cnt = A.tl.cnt[face];
                    const int64_t base = e * A.tl.elem + A.tl.face_off[face] + compact_index(vg, d, side, iv);
#pragma unroll
                    for (int fp = 0; fp < NFP; ++fp) {
                        Real t = Real(0);
#pragma unroll
                        for (int m = 0; m < N; ++m) t += (Real)A.ops.lam[side][m] * f[line_pt<N>(d, fp, m)];
                        trout[base + fp * cnt] = t;
                    }
                }
            }
        }

        // moments: transpose each wave's tile through LDS, lane = solution point
        if (A.do_moments) {
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                __syncthreads();
                if ((lane >> 5) == half) {
#pragma unroll
                    for (int s = 0; s < NS; ++s) tile[wave][s][lane & 31] = act ? f[s] : Real(0);
                }
                __syncthreads();
                if (lane < NS) {
                    const int kb = ch * kBlock + wave * 64 + half * 32;
                    const double *__restrict__ wp = A.wpsi + (int64_t)kb * NMOM;
#pragma unroll 4
                    for (int j = 0; j < 32; ++j) {
                        const double v = (double)tile[wave][lane][j];
#pragma unroll
                        for (int a = 0; a < NMOM; ++a) acc[a] += wp[j * NMOM + a] * v;
                    }
                }
            }
        }
    }

    if (A.do_moments) {
        __syncthreads();
        if (lane < NS) {
#pragma unroll
            for (int a = 0; a < NMOM; ++a) red[wave][lane][a] = acc[a];
        }
        __syncthreads();
        for (int i = tid; i < NS * NMOM; i += kBlock) {
            const int s = i / NMOM, a = i % NMOM;
            A.sa.Q[(e * NS + s) * NMOM + a] = ((red[0][s][a] + red[1][s][a]) + red[2][s][a]) + red[3][s][a];
        }
    }
}

template <typename Real, int P, int NMOM>
int launch_p(fr_dvm *h, int mode, const FrArgs &A) {
    dim3 grid((unsigned)h->ne), block(kBlock);
    if (mode == MODE_PRIME)
        hipLaunchKernelGGL((k_fr_axis<Real, P, NMOM, MODE_PRIME>), grid, block, 0, h->stream, A);
    else if (mode == MODE_STAGE)
        hipLaunchKernelGGL((k_fr_axis<Real, P, NMOM, MODE_STAGE>), grid, block, 0, h->stream, A);
    else
        hipLaunchKernelGGL((k_fr_axis<Real, P, NMOM, MODE_RESID>), grid, block, 0, h->stream, A);
    hipError_t st = hipGetLastError();
    if (st != hipSuccess) return h->fail(FR_DVM_EHIP, std::string("FR kernel launch: ") + hipGetErrorString(st));
    return FR_DVM_OK;
}

template <typename Real, int NMOM>
int launch_np(fr_dvm *h, int mode, const FrArgs &A) {
    switch (h->p) {
        case 1: return launch_p<Real, 1, NMOM>(h, mode, A);
        case 2: return launch_p<Real, 2, NMOM>(h, mode, A);
        case 3: return launch_p<Real, 3, NMOM>(h, mode, A);
    }
    return h->fail(FR_DVM_EUNSUPPORTED, "order");
}

}  // namespace

int launch_fr_axis(fr_dvm *h, int mode, const StageArgs &sa, int do_traces, int do_moments) {
    FrArgs A;
    A.ops = h->ops;
    A.vg = h->vg;
    A.tl = h->tl;
    A.ne = h->ne;
    A.nu = h->vg.nu;
    A.gfac = h->d_gfac;
    A.nbr = h->d_nbr;
    A.wpsi = h->d_wpsi;
    A.sa = sa;
    A.do_traces = do_traces;
    A.do_moments = do_moments;
    const bool fp64 = h->prm.precision == FR_DVM_FP64;
    if (h->nmom == 5)
        return fp64 ? launch_np<double, 5>(h, mode, A) : launch_np<float, 5>(h, mode, A);
    return fp64 ? launch_np<double, 10>(h, mode, A) : launch_np<float, 10>(h, mode, A);
}

}  // namespace frdvm
