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
// Work decomposition: one workgroup (4 wave64) per element.  A lane owns one
// velocity node and one z-layer of the element's N^3 Gauss points (N = p+1):
// N lanes share a velocity, a wave covers 64/N velocities.  On a
// tensor-product Gauss element every operator factorises along lines, so the
// x and y derivatives, traces and corrections are local to the lane's layer;
// z lines are gathered from a per-wave LDS tile that holds the wave's
// N^3 x (64/N) block of f.  The same tile, refilled with the stage result,
// serves the z traces of the result and the moment reduction (lane = solution
// point, FP64 accumulation with wave-uniform scalar weights, fixed order:
// bitwise reproducible).  Everything is VALU FMA: the factorised contractions
// have K = p+1 <= 4 and the kernel is HBM bound.
//
// Traces: each element stores, for the velocities leaving it through a face,
// its trace on that face ("outflow half", compact layout) into the trace
// buffer of the next stage; the downwind neighbour reads exactly those
// entries as its exterior state.  Two trace buffers alternate between stages.
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

// The LDS tile region of a wave is private to that wave, and one wave's LDS
// operations complete in issue order, so exchanging data through it only
// needs the compiler kept from moving LDS accesses across this point.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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
__global__ __launch_bounds__(kBlock) void k_fr_layer(const FrArgs A) {
    constexpr int N = P + 1, NS = N * N * N, NL = N * N;
    constexpr int VPW = 64 / N;       // velocities per wave
    constexpr int VPB = 4 * VPW;      // velocities per workgroup and chunk
    constexpr int TLD = VPW + 1;      // padded tile row
    __shared__ double s_eq[(MODE == MODE_STAGE) ? NS * kEqW : 1];
    constexpr size_t TILE_BYTES = sizeof(Real) * 4 * NS * TLD;
    constexpr size_t RED_BYTES = sizeof(double) * 4 * NS * NMOM;
    __shared__ __attribute__((aligned(16))) unsigned char s_raw[TILE_BYTES > RED_BYTES ? TILE_BYTES : RED_BYTES];
    Real(*tile)[NS][TLD] = reinterpret_cast<Real(*)[NS][TLD]>(s_raw);
    double(*red)[NS][NMOM] = reinterpret_cast<double(*)[NS][NMOM]>(s_raw);

    const int64_t e = blockIdx.x;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lay = lane / VPW;        // z-layer owned by this lane (N for an idle lane)
    const int vl = lane - lay * VPW;   // velocity slot inside the wave
    const bool lane_ok = lay < N;
    const int l = lane_ok ? lay : 0;
    const VGrid &vg = A.vg;
    const int nu = A.nu;
    const int64_t ebase = e * (int64_t)NS * nu;

    if (MODE == MODE_STAGE && A.sa.collide) {
        for (int i = tid; i < NS * kEqW; i += kBlock) s_eq[i] = A.sa.eq[e * NS * kEqW + i];
    }

    // z-direction operator entries of this lane's layer
    Real Dz[N], corrz[2];
#pragma unroll
    for (int m = 0; m < N; ++m) Dz[m] = (Real)A.ops.D[l * N + m];
    corrz[0] = (Real)A.ops.corr[0][l];
    corrz[1] = (Real)A.ops.corr[1][l];
    const double gf[3] = {A.gfac[3 * e], A.gfac[3 * e + 1], A.gfac[3 * e + 2]};

    double acc[NMOM];
#pragma unroll
    for (int a = 0; a < NMOM; ++a) acc[a] = 0.0;

    const Real *__restrict__ fin = reinterpret_cast<const Real *>(A.sa.f) + ebase + (int64_t)l * NL * nu;
    const Real *__restrict__ trin = reinterpret_cast<const Real *>(A.sa.tr_in);
    Real *__restrict__ trout = reinterpret_cast<Real *>(A.sa.tr_out);
    const int nchunk = (nu + VPB - 1) / VPB;
    __syncthreads();

    // stage value of the first chunk; later chunks are prefetched one ahead
    Real fnx[NL];
    {
        const int k0 = wave * VPW + vl;
        const bool a0 = lane_ok && k0 < nu;
#pragma unroll
        for (int q = 0; q < NL; ++q) fnx[q] = a0 ? fin[(int64_t)q * nu + k0] : Real(0);
    }

    for (int ch = 0; ch < nchunk; ++ch) {
        const int k = ch * VPB + wave * VPW + vl;
        const bool act = lane_ok && k < nu;
        const int kk = act ? k : 0;
        Real f[NL];
#pragma unroll
        for (int q = 0; q < NL; ++q) f[q] = fnx[q];
        {
            const int k1 = k + VPB;
            const bool a1 = lane_ok && k1 < nu;
#pragma unroll
            for (int q = 0; q < NL; ++q) fnx[q] = a1 ? fin[(int64_t)q * nu + k1] : Real(0);
        }
        int iv[3];
        iv[0] = kk % vg.nv[0];
        iv[1] = (kk / vg.nv[0]) % vg.nv[1];
        iv[2] = kk / (vg.nv[0] * vg.nv[1]);
        // The sign of each velocity component is taken from the integer split
        // of the grid computed on the host (not from the rounded value), so
        // the compact trace slots of writer and reader always agree; a node
        // classified as zero carries exactly zero flux.
        double u[3];
        int sgn[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            sgn[d] = iv[d] >= vg.pos_start[d] ? 1 : (iv[d] < vg.neg_end[d] ? -1 : 0);
            u[d] = sgn[d] == 0 ? 0.0 : __dadd_rn(vg.umin[d], __dmul_rn((double)iv[d], vg.du[d]));
        }

        if (MODE != MODE_PRIME) {
            // publish the stage value for the z-line gathers
            wave_sync();
            if (lane_ok) {
#pragma unroll
                for (int q = 0; q < NL; ++q) tile[wave][l * NL + q][vl] = f[q];
            }
            wave_sync();
            Real r[NL];
#pragma unroll
            for (int q = 0; q < NL; ++q) r[q] = Real(0);
            const Real ax = (Real)(gf[0] * u[0]), ay = (Real)(gf[1] * u[1]), az = (Real)(gf[2] * u[2]);
            // x and y derivatives inside the layer
#pragma unroll
            for (int j = 0; j < N; ++j)
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    Real tx = Real(0), ty = Real(0);
#pragma unroll
                    for (int m = 0; m < N; ++m) {
                        tx += (Real)A.ops.D[i * N + m] * f[m + N * j];
                        ty += (Real)A.ops.D[j * N + m] * f[i + N * m];
                    }
                    r[i + N * j] += ax * tx + ay * ty;
                }
            // z lines: derivative and the inflow correction of the z faces
            const int zin = sgn[2] > 0 ? 0 : 1;
            const bool zflow = act && sgn[2] != 0;
            int64_t zbase = 0, zcnt = 0;
            Real unz = Real(0);
            if (zflow) {
                const int nface = 4 + (zin ^ 1);
                zcnt = A.tl.cnt[nface];
                zbase = (int64_t)A.nbr[6 * e + 4 + zin] * A.tl.elem + A.tl.face_off[nface] + compact_index(vg, 2, zin ^ 1, iv);
                unz = (Real)((zin ? 1.0 : -1.0) * gf[2] * u[2]);
            }
#pragma unroll
            for (int q = 0; q < NL; ++q) {
                Real g[N];
#pragma unroll
                for (int m = 0; m < N; ++m) g[m] = tile[wave][m * NL + q][vl];
                Real t = Real(0);
#pragma unroll
                for (int m = 0; m < N; ++m) t += Dz[m] * g[m];
                r[q] += az * t;
                if (zflow) {
                    Real fm = Real(0);
#pragma unroll
                    for (int m = 0; m < N; ++m) fm += (Real)A.ops.lam[zin][m] * g[m];
                    const Real fp = trin[zbase + q * zcnt];
                    r[q] += corrz[zin] * (unz * (fp - fm));
                }
            }
            // x faces: face points (j, l); y faces: face points (i, l)
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                if (act && sgn[d] != 0) {
                    const int sin_ = sgn[d] > 0 ? 0 : 1;
                    const int nface = 2 * d + (sin_ ^ 1);
                    const int64_t cnt = A.tl.cnt[nface];
                    const int64_t base = (int64_t)A.nbr[6 * e + 2 * d + sin_] * A.tl.elem + A.tl.face_off[nface] +
                                         compact_index(vg, d, sin_ ^ 1, iv);
                    const Real un = (Real)((sin_ ? 1.0 : -1.0) * gf[d] * u[d]);
#pragma unroll
                    for (int a = 0; a < N; ++a) {
                        const Real fp = trin[base + (a + N * l) * cnt];
                        Real fm = Real(0);
#pragma unroll
                        for (int m = 0; m < N; ++m)
                            fm += (Real)A.ops.lam[sin_][m] * (d == 0 ? f[m + N * a] : f[a + N * m]);
                        const Real jmp = un * (fp - fm);
#pragma unroll
                        for (int m = 0; m < N; ++m)
                            r[d == 0 ? m + N * a : a + N * m] += (Real)A.ops.corr[sin_][m] * jmp;
                    }
                }
            }
            Real *__restrict__ out = reinterpret_cast<Real *>(A.sa.fout) + ebase + (int64_t)l * NL * nu;
            if (MODE == MODE_RESID) {
                if (act) {
#pragma unroll
                    for (int q = 0; q < NL; ++q) out[(int64_t)q * nu + k] = -r[q];
                }
                continue;
            }
            // collision source and the Runge-Kutta combination, point by point
            const Real *__restrict__ fnp = reinterpret_cast<const Real *>(A.sa.fn) + ebase + (int64_t)l * NL * nu;
            Real *__restrict__ dF = reinterpret_cast<Real *>(A.sa.dF) + ebase + (int64_t)l * NL * nu;
            const Real dt = (Real)A.sa.dt;
#pragma unroll
            for (int q = 0; q < NL; ++q) {
                Real L = -r[q];
                if (A.sa.collide) {
                    const double *eq = &s_eq[(l * NL + q) * kEqW];
                    const Real gq = eval_g<Real>(eq, u);
                    L += (gq - f[q]) * (Real)eq[EQ_INVTAU];
                }
                Real fo;
                if (A.sa.scheme == 0) {
                    fo = (Real)A.sa.beta * (f[q] + dt * L);
                    if (A.sa.alpha != 0.0 && act) fo += (Real)A.sa.alpha * fnp[(int64_t)q * nu + k];
                } else {
                    Real dd = dt * L;
                    if (A.sa.lsA != 0.0 && act) dd += (Real)A.sa.lsA * dF[(int64_t)q * nu + k];
                    if (act) dF[(int64_t)q * nu + k] = dd;
                    fo = f[q] + (Real)A.sa.lsB * dd;
                }
                f[q] = act ? fo : Real(0);
                if (act) out[(int64_t)q * nu + k] = fo;
            }
        }

        // outflow traces of the produced value on the x and y faces
        if (A.do_traces && act) {
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                if (sgn[d] != 0) {
                    const int side = sgn[d] > 0 ? 1 : 0;
                    const int face = 2 * d + side;
                    const int64_t cnt = A.tl.cnt[face];
                    const int64_t base = e * A.tl.elem + A.tl.face_off[face] + compact_index(vg, d, side, iv);
#pragma unroll
                    for (int a = 0; a < N; ++a) {
                        Real t = Real(0);
#pragma unroll
                        for (int m = 0; m < N; ++m)
                            t += (Real)A.ops.lam[side][m] * (d == 0 ? f[m + N * a] : f[a + N * m]);
                        trout[base + (a + N * l) * cnt] = t;
                    }
                }
            }
        }

        // tile of the produced value: z traces and the moment reduction
        if (A.do_moments || A.do_traces) {
            wave_sync();
            if (lane_ok) {
#pragma unroll
                for (int q = 0; q < NL; ++q) tile[wave][l * NL + q][vl] = f[q];
            }
            wave_sync();
            if (A.do_traces && act && sgn[2] != 0) {
                // this lane writes the z-face points (i, j = l)
                const int side = sgn[2] > 0 ? 1 : 0;
                const int face = 4 + side;
                const int64_t cnt = A.tl.cnt[face];
                const int64_t base = e * A.tl.elem + A.tl.face_off[face] + compact_index(vg, 2, side, iv);
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    const int q = i + N * l;
                    Real t = Real(0);
#pragma unroll
                    for (int m = 0; m < N; ++m) t += (Real)A.ops.lam[side][m] * tile[wave][m * NL + q][vl];
                    trout[base + q * cnt] = t;
                }
            }
            if (A.do_moments && lane < NS) {
                const int kb = ch * VPB + wave * VPW;
                const double *__restrict__ wp = A.wpsi + (int64_t)kb * NMOM;
#pragma unroll 4
                for (int j = 0; j < VPW; ++j) {
                    const double v = (double)tile[wave][lane][j];
#pragma unroll
                    for (int a = 0; a < NMOM; ++a) acc[a] += wp[j * NMOM + a] * v;
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
        hipLaunchKernelGGL((k_fr_layer<Real, P, NMOM, MODE_PRIME>), grid, block, 0, h->stream, A);
    else if (mode == MODE_STAGE)
        hipLaunchKernelGGL((k_fr_layer<Real, P, NMOM, MODE_STAGE>), grid, block, 0, h->stream, A);
    else
        hipLaunchKernelGGL((k_fr_layer<Real, P, NMOM, MODE_RESID>), grid, block, 0, h->stream, A);
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

// Streaming copy with 16-byte accesses, grid-stride.
__global__ __launch_bounds__(256) void k_copy16(uint4 *__restrict__ dst, const uint4 *__restrict__ src, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
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

extern "C" int fr_dvm_hbm_copy(void *dst, const void *src, size_t nbytes, void *stream) {
    if (!dst || !src || nbytes % 16 != 0) return FR_DVM_EINVAL;
    const char *d = static_cast<const char *>(dst), *s = static_cast<const char *>(src);
    if (d < s + nbytes && s < d + nbytes) return FR_DVM_EINVAL;
    int64_t n = (int64_t)(nbytes / 16);
    if (n == 0) return FR_DVM_OK;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 256 * 64) blocks = 256 * 64;
    hipLaunchKernelGGL(frdvm::k_copy16, dim3((unsigned)blocks), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                       static_cast<uint4 *>(dst), static_cast<const uint4 *>(src), n);
    return hipGetLastError() == hipSuccess ? FR_DVM_OK : FR_DVM_EHIP;
}
