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
// Work decomposition: one workgroup per element, one wave64 per z-layer of
// the element's N^3 Gauss points (N = p+1), one lane per velocity node: the
// velocity axis is walked in chunks of 64 nodes, so every access to f, the
// RK registers and the traces is a run of 64 consecutive velocities (256 B
// in FP32) per solution point.  On a tensor-product Gauss element every
// operator factorises along lines: the x and y lines lie in the lane's own
// layer; z lines cross the layers and are read from a workgroup LDS tile of
// the chunk's stage value.  A second tile takes the produced value for the z
// traces and the moment reduction (lane = solution point, FP64 accumulation
// with scalar-cache weights, fixed order: bitwise reproducible).  The
// equilibrium record of a point is uniform over a wave and is read through
// the scalar cache.  Everything is VALU FMA: the factorised contractions
// have K = p+1 <= 4 and the kernel is HBM bound.
//
// Latency: every HBM read of chunk c+1 (stage value, inflow traces) is
// issued while chunk c is computed, the second RK register of chunk c at
// its start.
//
// Traces: for the velocities leaving an element through a face, the element
// writes its trace on that face ("outflow half", compact layout) into the
// neighbour's block of the next stage's trace buffer, so each element reads
// its exterior states from its own block.  Two trace buffers alternate
// between stages.
//
// Reduced pair (F, G) (Section "Governing equations", moment records of 6 or
// 11 values): the chunk loop runs over F's velocities, then G's; each
// component has its own half of the element's trace block.  G relaxes to
// delta theta / 2 times F's equilibrium (its exponent shifted by the log of
// that factor) and adds only its integral to the moments.
#include <hip/hip_runtime.h>

#include <cstring>

#include "frdvm_common.h"
#include "frdvm_dev.h"

namespace frdvm {

namespace {

constexpr int MODE_PRIME = 0, MODE_STAGE = 1, MODE_RESID = 2;
constexpr int kChunk = 64;  // velocities per chunk: one per lane of a wave

// Register targets (waves per SIMD) of the stage kernel.  FP32: the LDS of a
// workgroup (48 KB at p = 3 with the ES moments) admits three workgroups of
// four waves per CU, i.e. 3 waves/SIMD; a target above what LDS admits is
// not honoured and leaves the kernel at 2.  FP64: LDS admits two.
#ifndef FRDVM_WAVES_F32
#define FRDVM_WAVES_F32 3
#endif
#ifndef FRDVM_WAVES_F64
#define FRDVM_WAVES_F64 2
#endif

// FR operators in the working precision of the kernel.
template <typename Real>
struct OpsR {
    Real D[kMaxN * kMaxN];
    Real lam[2][kMaxN];
    Real corr[2][kMaxN];
};

struct FrArgs {
    OpsR<float> of;
    OpsR<double> od;
    VGrid vg;
    TraceLayout tl;
    float inv_nx, inv_nxy;  // 1/nv_x and 1/(nv_x nv_y) for the index split
    int nu;
    const double *gfac;     // [ne][3]
    const int32_t *nbr;     // [ne][6]
    const double *wx3;      // [nv_x][3] moment weights along x
    const double *wrow;     // [nv_y nv_z][6] moment weights of a (y, z) row
    StageArgs sa;
    int do_traces, do_moments;
    int64_t elem_comp;   // trace entries of one component in an element block
    const double *gfp;   // [npts] the pair's G factor delta theta / 2 (records of 6 / 11)
};

template <typename Real>
__device__ __forceinline__ const OpsR<Real> &ops_of(const FrArgs &A);
template <>
__device__ __forceinline__ const OpsR<float> &ops_of<float>(const FrArgs &A) { return A.of; }
template <>
__device__ __forceinline__ const OpsR<double> &ops_of<double>(const FrArgs &A) { return A.od; }

// exp of an exponent held in FP64, returned in the working precision (FP32:
// evaluated in FP64 and rounded once, see exp_to_f32).
template <typename Real>
__device__ __forceinline__ Real exp_r(double E);
template <>
__device__ __forceinline__ float exp_r<float>(double E) {
    return exp_to_f32(E);
}
template <>
__device__ __forceinline__ double exp_r<double>(double E) {
    return exp_f64(E);
}

// Coefficient c (in the order of ref_exponent) of the exponent of an
// equilibrium record, c0 - (u-V)^T B (u-V)/2, as a polynomial in u.
__device__ __forceinline__ double ref_coef(const double *q, int c) {
    const double Bxx = q[EQ_B], Byy = q[EQ_B + 1], Bzz = q[EQ_B + 2];
    const double Bxy = q[EQ_B + 3], Bxz = q[EQ_B + 4], Byz = q[EQ_B + 5];
    const double Vx = q[EQ_V], Vy = q[EQ_V + 1], Vz = q[EQ_V + 2];
    const double bx = Bxx * Vx + Bxy * Vy + Bxz * Vz;  // B V: the linear coefficients
    const double by = Bxy * Vx + Byy * Vy + Byz * Vz;
    const double bz = Bxz * Vx + Byz * Vy + Bzz * Vz;
    switch (c) {
        case 0: return q[EQ_C0] - 0.5 * (Vx * bx + Vy * by + Vz * bz);
        case 1: return bx;
        case 2: return by;
        case 3: return bz;
        case 4: return -0.5 * Bxx;
        case 5: return -0.5 * Byy;
        case 6: return -0.5 * Bzz;
        case 7: return -Bxy;
        case 8: return -Bxz;
        default: return -Byz;
    }
}

// The exponent of a staged record at velocity u: the polynomial of
// ref_exponent with the constant term c0 given.
__device__ __forceinline__ double eq_exponent(const double *c, double c0, const double u[3]) {
    double tx = fma(c[4], u[0], c[1]);
    tx = fma(c[7], u[1], tx);
    tx = fma(c[8], u[2], tx);
    double ty = fma(c[5], u[1], c[2]);
    ty = fma(c[9], u[2], ty);
    const double tz = fma(c[6], u[2], c[3]);
    double E = fma(u[0], tx, c0);
    E = fma(u[1], ty, E);
    return fma(u[2], tz, E);
}


// Element-relative access: `base` is uniform (one element's slab), `boff`
// the lane's byte offset inside it (a slab stays below 4 GiB: at most
// 64 solution points x 2 components x 64^3 velocities x 8 bytes).
template <typename T>
__device__ __forceinline__ T ldb(const T *base, uint32_t boff) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + boff);
}
template <typename T>
__device__ __forceinline__ void stb(T *base, uint32_t boff, T v) {
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + boff) = v;
}
// The same with the non-temporal hint, for the state streams (f, the second
// RK register, the result): each value is touched once per launch and the
// slabs far exceed the caches, so nothing is kept for reuse (about 2 % off
// the FP32 stage and 4 % off the FP64 one at 24^3 / p = 3 / 20^3; the same
// hint on the trace streams and on the general-mesh kernels changed
// nothing measurable).
template <typename T>
__device__ __forceinline__ T ldn(const T *base, uint32_t boff) {
    return __builtin_nontemporal_load(reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + boff));
}
template <typename T>
__device__ __forceinline__ void stn(T *base, uint32_t boff, T v) {
    __builtin_nontemporal_store(v, reinterpret_cast<T *>(reinterpret_cast<char *>(base) + boff));
}

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

// Small tables a lane chooses from by its own velocity (operator rows of the
// inflow or outflow side, trace layout of a face, neighbour block) live in
// LDS and are read with per-lane addresses.  A select between two uniform
// values would need one of them copied into a vector register (one scalar
// operand per VALU instruction), and those copies stay live for the whole
// kernel.
template <typename Real>
struct LdsTab {
    Real lam[2][kMaxN], corr[2][kMaxN];
    Real D[kMaxN * kMaxN];  // read with a wave-uniform address (z lines)
    int64_t nb[6];     // element offset of each neighbour's trace block
    uint32_t cnt[6];   // trace entries per face point of each face slot
    uint32_t fo[6];    // offset of each face slot inside a block
};

// The velocity node a lane works on in one chunk.
struct Vel {
    int k;  // node index (the last node for a lane past the end of the grid)
    bool act;  // a node of the grid (false: the lane duplicates the last one)
    int iv[3];
    int sgn[3];
    double u[3];
};

template <bool B>
struct BoolC {
    static constexpr bool value = B;
};

__device__ __forceinline__ Vel velocity(const FrArgs &A, int k, bool lane_ok) {
    const VGrid &vg = A.vg;
    Vel v;
    v.act = lane_ok && k < A.nu;
    v.k = v.act ? k : A.nu - 1;
    // integer split through single precision; exact for node counts below
    // 2^21 (enforced at set-up): (k + 1/2)/n stays 1/(2n) away from integers
    const int nx = vg.nv[0], nxy = vg.nv[0] * vg.nv[1];
    const int i2 = (int)(((float)v.k + 0.5f) * A.inv_nxy);
    const int r2 = v.k - i2 * nxy;
    const int i1 = (int)(((float)r2 + 0.5f) * A.inv_nx);
    v.iv[0] = r2 - i1 * nx;
    v.iv[1] = i1;
    v.iv[2] = i2;
    // The sign of each component comes from the integer split of the grid
    // made on the host (not from the rounded value), so the compact trace
    // slots of writer and reader always agree; a node classified as zero
    // carries exactly zero flux.
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        v.sgn[d] = v.iv[d] >= vg.pos_start[d] ? 1 : (v.iv[d] < vg.neg_end[d] ? -1 : 0);
        v.u[d] = v.sgn[d] == 0 ? 0.0 : __dadd_rn(vg.umin[d], __dmul_rn((double)v.iv[d], vg.du[d]));
    }
    return v;
}

// Traces are pushed: an element writes the trace of each velocity leaving
// it through a face into the block of the neighbour across that face, under
// the slot of that face (compact layout of the outflow side).  The reader
// therefore finds all its inflow traces inside its own block: slot
// 2d + (s ^ 1) for inflow through its face (d, s).  `TraceOff` is the lane's
// byte offset of face point `fp0` in that block and the byte stride between
// face points; a lane without inflow (idle, or a zero component) reads the
// first entry of the block with stride 0 and ignores it.
struct TraceOff {
    uint32_t off, stride;
};

template <typename Real>
__device__ __forceinline__ TraceOff trace_in(const FrArgs &A, const LdsTab<Real> &T, const Vel &v, int d, int fp0) {
    TraceOff t;
    const bool flow = v.sgn[d] != 0;  // (a lane past the end reads what the last node reads)
    const int sin_ = v.sgn[d] > 0 ? 0 : 1;  // inflow face side
    const int slot = 2 * d + (sin_ ^ 1);     // the upwind neighbour's outflow face
    const uint32_t cnt = T.cnt[slot], fo = T.fo[slot];
    const uint32_t idx = fo + (uint32_t)compact_index(A.vg, d, sin_ ^ 1, v.iv) +
                         (uint32_t)fp0 * cnt;
    t.off = flow ? idx * (uint32_t)sizeof(Real) : 0u;
    t.stride = flow ? cnt * (uint32_t)sizeof(Real) : 0u;
    return t;
}

// A value the compiler cannot see through (nor hoist out of a loop).
__device__ __forceinline__ int opaque(int x) {
    asm volatile("" : "+v"(x));
    return x;
}

// Keeps the compiler from moving memory accesses (and the scheduler from
// moving anything) across this point: bounds how many LDS values are in
// registers at once.
__device__ __forceinline__ void phase_fence() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

// Pins a value in a register at this point (its computation can be neither
// sunk below nor rematerialised after it).
template <typename T>
__device__ __forceinline__ void keep(T &x) {
    asm volatile("" : "+v"(x));
}

// Waves per SIMD the register allocation is held to (the prime pass keeps
// little state and is given more).
template <typename Real, int MODE>
constexpr int fr_waves() {
    return MODE == MODE_PRIME ? 4 : (sizeof(Real) == 4 ? FRDVM_WAVES_F32 : FRDVM_WAVES_F64);
}

// LDS tiles: one row of kChunk velocities per solution point, padded by one
// element so that the moment pass (lane = solution point, reading along its
// row) hits distinct banks; written and read elsewhere with lane = velocity.
constexpr int kTileLd = kChunk + 1;
template <typename Real>
__device__ __forceinline__ int tix(int row, int col) {
    return row * kTileLd + col;
}

typedef const __attribute__((address_space(4))) double cdouble;

// Real: arithmetic, LDS tiles and traces; SReal: storage of the state, the
// second RK register and the output.  ER (FP32 deviation storage, stage
// mode, FP32): the stage value and the inflow traces arrive as FP32
// deviations from element references and the result leaves as one.
template <typename Real, typename SReal, int P, int NMOM, int MODE, bool ER>
__global__ __launch_bounds__(kChunk *(P + 1)) __attribute__((amdgpu_waves_per_eu(fr_waves<Real, MODE>()))) void
k_fr_layer(const FrArgs A) {
    constexpr int N = P + 1, NS = N * N * N, NL = N * N;
    constexpr int NT = kChunk * N;                  // threads: one wave per z-layer
    constexpr int VPM = (kChunk + N - 1) / N;       // chunk velocities per wave in the moment pass
    constexpr bool FLUX = MODE != MODE_PRIME;
    constexpr bool STAGE = MODE == MODE_STAGE;
    // moment records of 6 / 11 values: the reduced pair (F, G), per point F
    // then G (nu values each); G is advected like F, relaxes to delta theta /
    // 2 times F's equilibrium and adds only its integral to the moments
    constexpr int NCOMP = (NMOM == 6 || NMOM == 11) ? 2 : 1;
    // the chunk's stage value (all layers, for the z lines) and z-face inflow
    // traces; the produced value (for the z traces and the moments).  The
    // prime pass uses the two value tiles alternately, chunk by chunk.  The
    // moment partial sums of the waves reuse the tiles after the loop.
    constexpr int TS = NS * kTileLd, TZ_ = FLUX ? NL * kTileLd : 1, TP = NS * kTileLd;
    constexpr int TBYTES = (TS + TZ_ + TP) * (int)sizeof(Real);
    constexpr int RBYTES = N * NS * NMOM * (int)sizeof(double);
    __shared__ __attribute__((aligned(16))) char s_tiles[TBYTES > RBYTES ? TBYTES : RBYTES];
    Real *const tS = reinterpret_cast<Real *>(s_tiles);
    Real *const tZ = tS + TS;
    Real *const tP = tZ + TZ_;
    double *const red = reinterpret_cast<double *>(s_tiles);
    __shared__ __attribute__((aligned(16))) LdsTab<Real> T;
    // equilibrium records staged per workgroup: the exponent as a polynomial
    // in u (10 coefficients), the G exponent shift (reduced pair), and 1/tau
    // in the working precision, read with a wave-uniform address
    constexpr bool EQ_LDS = STAGE;
    constexpr int kEb = 12;
    __shared__ __attribute__((aligned(16))) double s_eb[EQ_LDS ? NS * kEb : 1];
    __shared__ __attribute__((aligned(16))) Real s_it[EQ_LDS ? NS : 1];

    const OpsR<Real> &op = ops_of<Real>(A);
    const int64_t e = A.sa.e0 + blockIdx.x;
    const int tid = threadIdx.x;
    const int vl = tid & (kChunk - 1);                       // velocity of the chunk (lane)
    const int l = __builtin_amdgcn_readfirstlane(tid >> 6);  // z-layer of the wave
    const int nu = A.nu;
    const int64_t ebase = e * (int64_t)NS * nu * NCOMP;
    const uint32_t lrow = (uint32_t)(l * NL) * (uint32_t)(nu * NCOMP);  // offset of the layer inside the element
    const uint32_t QB = (uint32_t)(nu * NCOMP) * (uint32_t)sizeof(SReal);  // bytes between solution points
    // FP32 deviation storage: the element references of the previous stage's
    // records (own, and the neighbour across each face: the inflow traces are
    // deviations from the writer's) and of this stage's (own: the result)
    static_assert(!ER || (sizeof(Real) == 4 && sizeof(SReal) == 4 && MODE == MODE_STAGE && NCOMP == 1),
                  "deviation storage: FP32 monatomic stage kernel");
    const bool in_dev = ER && A.sa.in_dev;
    const bool out_dev = ER && A.sa.out_dev;
    // own prev, own cur, 6 faces' prev, own reference of the step's initial value (SSP)
    __shared__ __attribute__((aligned(16))) float s_ref[ER ? 9 * kRefCoef : 1];
    if (ER) {
        for (int t = tid; t < 9 * kRefCoef; t += NT) {
            const int r = t / kRefCoef;
            const int64_t er = (r < 2 || r == 8) ? e : (int64_t)A.nbr[6 * e + r - 2];
            const double *src = r == 1 ? A.sa.ref_cur : (r == 8 ? A.sa.ref_u0 : A.sa.ref_prev);
            s_ref[t] = (float)src[er * kRefW + t % kRefCoef];
        }
    }

    const bool collide = STAGE && A.sa.collide;
    if (EQ_LDS && collide) {
        for (int t = tid; t < NS * kEb; t += NT) {
            const int s = t / kEb, c = t % kEb;
            const double *q = A.sa.eq + (e * NS + s) * kEqW;
            double v = 0.0;
            if (c < kRefCoef) {
                v = ref_coef(q, c);
            } else if (c == kRefCoef) {
                if constexpr (NCOMP == 2) {
                    const double gf = A.gfp[e * NS + s];
                    v = gf > 0.0 ? log(gf) : -1000.0;  // the G exponent shift
                }
            } else {
                s_it[s] = (Real)q[EQ_INVTAU];
            }
            s_eb[t] = v;
        }
    }

    const double gf[3] = {A.gfac[3 * e], A.gfac[3 * e + 1], A.gfac[3 * e + 2]};
    // tables chosen from per lane (read only after the barrier below)
    if (tid < 2 * kMaxN) {
        const int sd = tid / kMaxN, m = tid % kMaxN;
        T.lam[sd][m] = op.lam[sd][m];
        T.corr[sd][m] = op.corr[sd][m];
    } else if (tid >= 64 && tid < 64 + kMaxN * kMaxN) {
        T.D[tid - 64] = op.D[tid - 64];
    } else if (tid < 2 * kMaxN + 6) {
        const int fc = tid - 2 * kMaxN;
        T.nb[fc] = (int64_t)A.nbr[6 * e + fc] * A.tl.elem;
        T.cnt[fc] = (uint32_t)A.tl.cnt[fc];
        T.fo[fc] = (uint32_t)A.tl.face_off[fc];
    }
    // trace blocks: the own one (inflow of this stage) and the neighbours'
    // (outflow of the produced value)
    const Real *__restrict__ trE = reinterpret_cast<const Real *>(A.sa.tr_in) + (FLUX ? e * A.tl.elem : 0);
    // running moments of the solution point tid % 64 over this wave's share
    // of every chunk (one partial per wave, added in wave order at the end)
    double Mrun[NMOM];
#pragma unroll
    for (int a = 0; a < NMOM; ++a) Mrun[a] = 0.0;
    // the lane tables (and the staged records) are complete from here on
    __syncthreads();

    const SReal *__restrict__ fE = reinterpret_cast<const SReal *>(A.sa.f) + ebase;
    Real *__restrict__ trout = reinterpret_cast<Real *>(A.sa.tr_out);
    SReal *__restrict__ outE = reinterpret_cast<SReal *>(A.sa.fout) + ebase;
    SReal *__restrict__ dFE = reinterpret_cast<SReal *>(A.sa.dF) + ebase;
    // second register read by the stage: f^n (SSP, alpha != 0) or dF (LSRK, A != 0)
    const bool useX = STAGE && (A.sa.scheme == 0 ? A.sa.alpha != 0.0 : A.sa.lsA != 0.0);
    const SReal *__restrict__ XE = STAGE ? (A.sa.scheme == 0 ? reinterpret_cast<const SReal *>(A.sa.fn) + ebase
                                                              : reinterpret_cast<const SReal *>(A.sa.dF) + ebase)
                                         : nullptr;
    const int nchunk = (nu + kChunk - 1) / kChunk;
    const int ntot = NCOMP * nchunk;  // chunks of all components, F first

    // The stage value and the inflow traces of chunk c+1 are requested while
    // chunk c is computed.  Of the z-face traces (N^2 points per velocity,
    // needed by every layer) the wave of layer l fetches the points (i, l)
    // and passes them on through the tile.
    SReal fc[NL];
    Real TX[N], TY[N], TZ[N];
    {
        const Vel v0 = velocity(A, vl, true);
        const uint32_t o = (lrow + (uint32_t)v0.k) * (uint32_t)sizeof(SReal);
#pragma unroll
        for (int q = 0; q < NL; ++q) fc[q] = ldn(fE, o + q * QB);
        if (FLUX) {
            const TraceOff sx = trace_in<Real>(A, T, v0, 0, N * l);
            const TraceOff sy = trace_in<Real>(A, T, v0, 1, N * l);
            const TraceOff sz = trace_in<Real>(A, T, v0, 2, N * l);
#pragma unroll
            for (int a = 0; a < N; ++a) {
                TX[a] = ldb(trE, sx.off + a * sx.stride);
                TY[a] = ldb(trE, sy.off + a * sy.stride);
                TZ[a] = ldb(trE, sz.off + a * sz.stride);
            }
        }
    }

    for (int cc = 0; cc < ntot; ++cc) {
        // the lane's tile column, recomputed every chunk: tile addresses are
        // then formed from it with immediate offsets instead of being kept
        // in registers across the loop
        const int vt = opaque(vl);
        const int comp = NCOMP == 2 && cc >= nchunk ? 1 : 0;
        const int ch = cc - comp * nchunk;
        const Vel v = velocity(A, ch * kChunk + vl, true);
        const uint32_t o = (lrow + (uint32_t)(comp * nu + v.k)) * (uint32_t)sizeof(SReal);
        // tile taking the stage value of the chunk, and tile read by the z
        // traces and the moment pass (the same, alternating, for the prime pass)
        Real *const tpub = FLUX ? tS : ((cc & 1) ? tP : tS);
        Real *const tout = FLUX ? tP : tpub;
        // Publish the stage value (the prime pass: into the tile its z traces
        // and moments read) and this wave's z-face traces; every later use of
        // the stage value reads the tile, so its registers take the next
        // chunk's loads right away.
        // The lane's element references at its velocity (FP32 deviation
        // storage): rp the previous stage's (the stage value and the traces
        // are made relative to it), sh what turns a result relative to rp
        // into one relative to this stage's reference rc (rp - rc; rp after
        // the call's last stage, which leaves the plain value), dl[d] what
        // turns the inflow trace of direction d (relative to its writer's
        // reference, or plain in the first stage) into one relative to rp.
        // References are FP32 numbers: the difference of two within a factor
        // 2 of each other is exact in FP32 (consecutive stages' references
        // of an element are), and rounded once otherwise.  SSP adds the
        // step's initial value fn (relative to its reference r0) with weight
        // alpha: shd = alpha r0 + beta rp - rc, in FP64.
        float rp = 0.0f, sh = 0.0f, dl[3] = {0.0f, 0.0f, 0.0f};
        double shd = 0.0;
        if (ER) {
            const float uf[3] = {(float)v.u[0], (float)v.u[1], (float)v.u[2]};
            rp = ref_value(ref_exponent(&s_ref[0], uf));
            const float rc = out_dev ? ref_value(ref_exponent(&s_ref[kRefCoef], uf)) : 0.0f;
            sh = rp - rc;
            if (A.sa.scheme == 0) {
                const double r0 = A.sa.fn_dev ? (double)ref_value(ref_exponent(&s_ref[8 * kRefCoef], uf)) : 0.0;
                shd = fma(A.sa.alpha, r0, fma(A.sa.beta, (double)rp, -(double)rc));
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int slot = 2 + 2 * d + (v.sgn[d] > 0 ? 0 : 1);  // the upwind neighbour in direction d
                const float rn = in_dev ? ref_value(ref_exponent(&s_ref[slot * kRefCoef], uf)) : 0.0f;
                dl[d] = rn - rp;
            }
        }
#pragma unroll
        for (int q = 0; q < NL; ++q)
            tpub[tix<Real>(l * NL + q, vt)] = (ER && !in_dev) ? (Real)fc[q] - (Real)rp : (Real)fc[q];
        if (FLUX) {
#pragma unroll
            for (int a = 0; a < N; ++a) tZ[tix<Real>(N * l + a, vt)] = ER ? TZ[a] + (Real)dl[2] : TZ[a];
        }
        // the second RK register of this chunk, requested before the next
        // chunk's values (loads complete in order: waiting for these in the
        // collision then leaves the next chunk's loads in flight) and before
        // the x/y/z passes, which cover its latency
        SReal X[NL];
        if (useX) {
#pragma unroll
            for (int q = 0; q < NL; ++q) X[q] = ldn(XE, o + q * QB);
        } else {
#pragma unroll
            for (int q = 0; q < NL; ++q) X[q] = SReal(0);
        }
        TraceOff nx{0u, 0u}, ny{0u, 0u};
        // the next chunk (possibly the first of the next component)
        const int compn = NCOMP == 2 && cc + 1 >= nchunk ? 1 : 0;
        const Real *__restrict__ trEn = trE + (NCOMP == 2 ? compn * A.elem_comp : 0);
        {
            const int chn = cc + 1 - compn * nchunk;
            const Vel vn = velocity(A, chn * kChunk + vl, NCOMP == 1 || cc + 1 < ntot);
            const uint32_t on = (lrow + (uint32_t)(compn * nu + vn.k)) * (uint32_t)sizeof(SReal);
#pragma unroll
            for (int q = 0; q < NL; ++q) fc[q] = ldn(fE, on + q * QB);
            if (FLUX) {
                nx = trace_in<Real>(A, T, vn, 0, N * l);
                ny = trace_in<Real>(A, T, vn, 1, N * l);
                const TraceOff nz = trace_in<Real>(A, T, vn, 2, N * l);
#pragma unroll
                for (int a = 0; a < N; ++a) TZ[a] = ldb(trEn, nz.off + a * nz.stride);
            }
        }
        if (FLUX) __syncthreads();  // the chunk's stage value of every layer is in the tile
        Real f[NL];  // the produced value (stage and residual modes)

        if (FLUX) {
            Real r[NL];
#pragma unroll
            for (int q = 0; q < NL; ++q) r[q] = Real(0);
            const Real ax = (Real)(gf[0] * v.u[0]), ay = (Real)(gf[1] * v.u[1]), az = (Real)(gf[2] * v.u[2]);
            // x lines (rows j) then y lines (columns i) of the layer: the
            // derivative and the inflow correction of the x / y faces
            // (face points (j, l) / (i, l))
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                const bool flow = v.sgn[d] != 0;
                const int sin_ = v.sgn[d] > 0 ? 0 : 1;
                const Real un = (Real)((sin_ ? 1.0 : -1.0) * gf[d] * v.u[d]);
                const Real ad = d == 0 ? ax : ay;
                const TraceOff sn = d == 0 ? nx : ny;
#pragma unroll
                for (int a = 0; a < N; ++a) {
                    Real g[N];
#pragma unroll
                    for (int m = 0; m < N; ++m) g[m] = tS[tix<Real>(l * NL + (d == 0 ? m + N * a : a + N * m), vt)];
                    Real fm = Real(0);
#pragma unroll
                    for (int m = 0; m < N; ++m) fm += T.lam[sin_][m] * g[m];
                    Real &tin = d == 0 ? TX[a] : TY[a];
                    const Real jmp = flow ? un * ((ER ? tin + (Real)dl[d] : tin) - fm) : Real(0);
                    tin = ldb(trEn, sn.off + a * sn.stride);
#pragma unroll
                    for (int i = 0; i < N; ++i) {
                        Real t = Real(0);
#pragma unroll
                        for (int m = 0; m < N; ++m) t += op.D[i * N + m] * g[m];
                        Real &ri = r[d == 0 ? i + N * a : a + N * i];
                        ri = fma(ad, t, ri);
                        ri = fma(T.corr[sin_][i], jmp, ri);
                        keep(ri);
                    }
                    phase_fence();
                }
            }
            // z lines: derivative and inflow correction of the z faces in one
            // pass over the layers, r += sum_m (az Dz[m] - cz lam[m]) f_m,
            // then r += cz f+ (the interior trace folded into the coefficients)
            {
                const int zin = v.sgn[2] > 0 ? 0 : 1;
                const bool zflow = v.sgn[2] != 0;
                const Real unz = (Real)((zin ? 1.0 : -1.0) * gf[2] * v.u[2]);
                const Real cz = zflow ? T.corr[zin][l] * unz : Real(0);
#pragma unroll
                for (int m = 0; m < N; ++m) {
                    const Real cm = az * T.D[l * N + m] - cz * T.lam[zin][m];
#pragma unroll
                    for (int q = 0; q < NL; ++q) {
                        r[q] = fma(cm, tS[tix<Real>(m * NL + q, vt)], r[q]);
                        keep(r[q]);
                    }
                    phase_fence();
                }
#pragma unroll
                for (int q = 0; q < NL; ++q) {
                    const Real fp = zflow ? tZ[tix<Real>(q, vt)] : Real(0);
                    r[q] = fma(cz, fp, r[q]);
                }
                phase_fence();
            }
            if (MODE == MODE_RESID) {
#pragma unroll
                for (int q = 0; q < NL; ++q) stn(outE, o + q * QB, (SReal)(-r[q]));
                __syncthreads();  // every layer is done with the stage tile
                continue;
            }
            // collision source and the Runge-Kutta combination, point by point
            const Real dt = (Real)A.sa.dt;
            // random bits of the stochastic rounding: one hash per lane and
            // chunk, a xorshift step per value
            uint32_t rs = sizeof(Real) == 4 ? round_bits(A.sa.seed, (uint32_t)(e * NS + l * NL), (uint32_t)(comp * nu + v.k)) | 1u
                                            : 0u;
            // One loop per combination of the launch-uniform switches (the
            // collision, the RK scheme, whether dF is kept), and lanes past
            // the end of the grid computing and storing exactly what the lane
            // of the last node does: no branch splits the points, so the
            // scheduler can interleave their independent chains.
            auto points = [&](auto coll_c, auto lsrk_c, auto keep_c) {
                constexpr bool COLL = decltype(coll_c)::value, LSRK = decltype(lsrk_c)::value;
                constexpr bool KEEP = decltype(keep_c)::value;
#pragma unroll
                for (int q = 0; q < NL; ++q) {
                    const Real fq = tS[tix<Real>(l * NL + q, vt)];
                    Real L = -r[q];
                    if constexpr (COLL) {
                        const int s = l * NL + q;
                        const double *b = &s_eb[s * kEb];
                        const double c0 = (NCOMP == 2 && comp) ? b[0] + b[kRefCoef] : b[0];
                        // the equilibrium's exponent at this point and velocity
                        const double Eq = eq_exponent(b, c0, v.u);
                        if constexpr (ER)
                            L += ((Real)(exp_f64(Eq) - (double)rp) - fq) * s_it[s];  // g - rp rounded once
                        else
                            L += (exp_r<Real>(Eq) - fq) * s_it[s];
                    }
                    // the result, in FP64 for the stochastic rounding of the FP32 state
                    double fod;
                    if constexpr (!LSRK) {
                        fod = A.sa.beta * ((double)fq + (double)(dt * L));
                        fod = fma(A.sa.alpha, (double)X[q], fod);  // (X = 0 when not read)
                    } else {
                        Real dd = dt * L;
                        dd += (Real)A.sa.lsA * (Real)X[q];
                        if constexpr (KEEP) stn(dFE, o + q * QB, (SReal)dd);
                        fod = fma(A.sa.lsB, (double)dd, (double)fq);
                    }
                    if constexpr (ER) fod += LSRK ? (double)sh : shd;
                    Real fo;
                    if constexpr (sizeof(Real) == 4) {
                        rs = xorshift32(rs);
                        fo = round_stochastic(fod, rs);
                    } else {
                        fo = (Real)fod;
                    }
                    f[q] = fo;
                    stn(outE, o + q * QB, (SReal)fo);
                    // (a fence every two points in FP32, four in FP64: the
                    // chains in flight at once, against register pressure)
                    if (q % (sizeof(Real) == 4 ? 2 : 4) == (sizeof(Real) == 4 ? 1 : 3)) phase_fence();
                }
            };
            if constexpr (STAGE) {
                if (A.sa.scheme == 0) {
                    if (collide) points(BoolC<true>{}, BoolC<false>{}, BoolC<false>{});
                    else points(BoolC<false>{}, BoolC<false>{}, BoolC<false>{});
                } else if (A.sa.keep_dF) {
                    if (collide) points(BoolC<true>{}, BoolC<true>{}, BoolC<true>{});
                    else points(BoolC<false>{}, BoolC<true>{}, BoolC<true>{});
                } else {
                    if (collide) points(BoolC<true>{}, BoolC<true>{}, BoolC<false>{});
                    else points(BoolC<false>{}, BoolC<true>{}, BoolC<false>{});
                }
            }
        }

        // outflow traces of the produced value on the x and y faces, into
        // the neighbours' blocks
        if (A.do_traces) {
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                if (v.sgn[d] != 0) {
                    const int side = v.sgn[d] > 0 ? 1 : 0;
                    const int face = 2 * d + side;
                    const int cnt = (int)T.cnt[face];
                    Real *tp = trout + T.nb[face] + (NCOMP == 2 ? comp * A.elem_comp : 0) + T.fo[face] +
                               compact_index(A.vg, d, side, v.iv) +
                               (int64_t)(N * l) * cnt;
#pragma unroll
                    for (int a = 0; a < N; ++a) {
                        Real t = Real(0);
                        if (FLUX) {
#pragma unroll
                            for (int m = 0; m < N; ++m)
                                t += T.lam[side][m] * (d == 0 ? f[m + N * a] : f[a + N * m]);
                        } else {
#pragma unroll
                            for (int m = 0; m < N; ++m)
                                t += T.lam[side][m] * tpub[tix<Real>(l * NL + (d == 0 ? m + N * a : a + N * m), vt)];
                        }
                        tp[a * cnt] = t;
                    }
                }
            }
        }

        // produced value of every layer: z traces and the moment reduction
        if (A.do_moments || A.do_traces) {
            if (FLUX) {
#pragma unroll
                for (int q = 0; q < NL; ++q) tP[tix<Real>(l * NL + q, vt)] = f[q];
            }
            __syncthreads();  // the produced tile is complete (and the stage tile no longer read)
            if (A.do_traces && v.sgn[2] != 0) {
                // this wave writes the z-face points (i, j = l)
                const int side = v.sgn[2] > 0 ? 1 : 0;
                const int face = 4 + side;
                const int cnt = (int)T.cnt[face];
                Real *tp = trout + T.nb[face] + (NCOMP == 2 ? comp * A.elem_comp : 0) + T.fo[face] +
                           compact_index(A.vg, 2, side, v.iv) +
                           (int64_t)(N * l) * cnt;
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    const int q = i + N * l;
                    Real t = Real(0);
#pragma unroll
                    for (int m = 0; m < N; ++m) t += T.lam[side][m] * tout[tix<Real>(m * NL + q, vt)];
                    tp[i * cnt] = t;
                }
            }
            if (A.do_moments && vl < NS) {
                // Moments of this wave's share of the chunk (lane = solution
                // point).  Along an x-row only w_x varies with the node; each
                // row segment is summed as (sum w_x f, sum w_x u_x f,
                // sum w_x u_x^2 f) and closed with the row's (y, z) weights:
                // 3 FMA per node instead of one per moment.  Weights are
                // wave-uniform and read through the scalar cache (never
                // written by the kernel).
                cdouble *wx3 = (cdouble *)A.wx3;
                cdouble *wrow = (cdouble *)A.wrow;
                const int j0 = l * VPM;
                const int kb = ch * kChunk + j0;
                const int nx = A.vg.nv[0];
                int jn = kChunk - j0 < VPM ? kChunk - j0 : VPM;
                if (nu - kb < jn) jn = nu - kb;
                int ix = kb % nx, row = kb / nx;
                double M[NMOM], a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
                for (int a = 0; a < NMOM; ++a) M[a] = 0.0;
                for (int j = 0; j < jn; ++j) {
                    const double x = (double)tout[tix<Real>(vt, j0 + j)];
                    a0 = fma(wx3[3 * ix], x, a0);
                    a1 = fma(wx3[3 * ix + 1], x, a1);
                    a2 = fma(wx3[3 * ix + 2], x, a2);
                    if (++ix == nx || j == jn - 1) {
                        cdouble *wr = wrow + 6 * row;
                        if (NCOMP == 2 && comp) {
                            // G: only its integral
                            M[NMOM - 1] = fma(wr[0], a0, M[NMOM - 1]);
                            a0 = a1 = a2 = 0.0;
                            if (ix == nx) {
                                ix = 0;
                                ++row;
                            }
                            continue;
                        }
                        M[0] = fma(wr[0], a0, M[0]);
                        M[1] = fma(wr[0], a1, M[1]);
                        M[2] = fma(wr[1], a0, M[2]);
                        M[3] = fma(wr[2], a0, M[3]);
                        if constexpr (NMOM == 5 || NMOM == 6) {
                            M[4] = fma(0.5, fma(wr[0], a2, (wr[3] + wr[4]) * a0), M[4]);
                        } else {
                            M[4] = fma(wr[0], a2, M[4]);
                            M[5] = fma(wr[3], a0, M[5]);
                            M[6] = fma(wr[4], a0, M[6]);
                            M[7] = fma(wr[1], a1, M[7]);
                            M[8] = fma(wr[2], a1, M[8]);
                            M[9] = fma(wr[5], a0, M[9]);
                        }
                        a0 = a1 = a2 = 0.0;
                        if (ix == nx) {
                            ix = 0;
                            ++row;
                        }
                    }
                }
#pragma unroll
                for (int a = 0; a < NMOM; ++a) Mrun[a] += M[a];
            }
        } else if (FLUX) {
            __syncthreads();  // every layer is done with the stage tile
        }
    }

    if (A.do_moments) {
        __syncthreads();  // the tiles are free: they take the waves' partial sums
        if (vl < NS) {
#pragma unroll
            for (int a = 0; a < NMOM; ++a) red[(l * NS + vl) * NMOM + a] = Mrun[a];
        }
        __syncthreads();
        for (int i = tid; i < NS * NMOM; i += NT) {
            double t = red[i];
#pragma unroll
            for (int w = 1; w < N; ++w) t += red[w * NS * NMOM + i];
            // (deviation storage: plus the moments of the element reference)
            A.sa.Q[(e * NS) * NMOM + i] = out_dev ? t + A.sa.ref_cur[e * kRefW + kRefCoef + i % NMOM] : t;
        }
    }
}

// Element reference of the FP32 deviation storage from the current
// equilibrium records: the exponent polynomial (ref_exponent) whose
// coefficients are the means over the element's solution points of the
// monomial coefficients of the points' equilibrium exponents
// c0 - (u-V)^T B (u-V)/2 (points without an equilibrium are left out; none
// left: the reference is 0), and the moments of the reference on the
// velocity grid with the moment pass's weights, in FP64 and a fixed order.
// One workgroup per element.
constexpr int kRefBlock = 256;
static_assert(kRefCoef + 10 <= kRefW, "element reference record: coefficients and up to 10 moments");


template <int NMOM>
__global__ __launch_bounds__(kRefBlock) void k_elem_ref(const FrArgs A, int ns, double *__restrict__ ref) {
    __shared__ double s_c[kRefCoef];
    __shared__ float s_cf[kRefCoef];  // the coefficients as the stage kernel reads them
    __shared__ double s_m[kRefBlock * NMOM];
    const int64_t e = blockIdx.x;
    const int tid = threadIdx.x;
    if (tid < kRefCoef) {
        double sum = 0.0;
        int cnt = 0;
        for (int s = 0; s < ns; ++s) {
            const double *q = A.sa.eq + (e * ns + s) * kEqW;
            if (!isfinite(q[EQ_C0])) continue;
            sum += ref_coef(q, tid);
            ++cnt;
        }
        s_c[tid] = cnt ? sum / cnt : (tid == 0 ? -INFINITY : 0.0);
        s_cf[tid] = (float)s_c[tid];
    }
    __syncthreads();
    double M[NMOM];
#pragma unroll
    for (int a = 0; a < NMOM; ++a) M[a] = 0.0;
    const int nx = A.vg.nv[0];
    for (int k = tid; k < A.nu; k += kRefBlock) {
        const Vel v = velocity(A, k, true);
        const float uf[3] = {(float)v.u[0], (float)v.u[1], (float)v.u[2]};
        const double r = (double)ref_value(ref_exponent(s_cf, uf));
        const double *wx = A.wx3 + 3 * (k % nx), *wr = A.wrow + 6 * (k / nx);
        const double a0 = wx[0] * r, a1 = wx[1] * r, a2 = wx[2] * r;
        M[0] = fma(wr[0], a0, M[0]);
        M[1] = fma(wr[0], a1, M[1]);
        M[2] = fma(wr[1], a0, M[2]);
        M[3] = fma(wr[2], a0, M[3]);
        if constexpr (NMOM == 5) {
            M[4] = fma(0.5, fma(wr[0], a2, (wr[3] + wr[4]) * a0), M[4]);
        } else {
            M[4] = fma(wr[0], a2, M[4]);
            M[5] = fma(wr[3], a0, M[5]);
            M[6] = fma(wr[4], a0, M[6]);
            M[7] = fma(wr[1], a1, M[7]);
            M[8] = fma(wr[2], a1, M[8]);
            M[9] = fma(wr[5], a0, M[9]);
        }
    }
#pragma unroll
    for (int a = 0; a < NMOM; ++a) s_m[tid * NMOM + a] = M[a];
    __syncthreads();
    double *out = ref + e * kRefW;
    if (tid < NMOM) {
        double t = 0.0;
        for (int i = 0; i < kRefBlock; ++i) t += s_m[i * NMOM + tid];
        out[kRefCoef + tid] = t;
    } else if (tid >= 64 && tid < 64 + kRefCoef) {
        out[tid - 64] = s_c[tid - 64];
    }
}

template <typename Real, typename SReal, int P, int NMOM, bool ER>
int launch_p(fr_dvm *h, int mode, const FrArgs &A) {
    dim3 grid((unsigned)(A.sa.ecount ? A.sa.ecount : h->ne)), block(kChunk * (P + 1));
    if (mode == MODE_PRIME)
        hipLaunchKernelGGL((k_fr_layer<Real, SReal, P, NMOM, MODE_PRIME, false>), grid, block, 0, h->stream, A);
    else if (mode == MODE_STAGE)
        hipLaunchKernelGGL((k_fr_layer<Real, SReal, P, NMOM, MODE_STAGE, ER>), grid, block, 0, h->stream, A);
    else
        hipLaunchKernelGGL((k_fr_layer<Real, SReal, P, NMOM, MODE_RESID, false>), grid, block, 0, h->stream, A);
    hipError_t st = hipGetLastError();
    if (st != hipSuccess) return h->fail(FR_DVM_EHIP, std::string("FR kernel launch: ") + hipGetErrorString(st));
    return FR_DVM_OK;
}

template <typename Real, typename SReal, int NMOM, bool ER = false>
int launch_np(fr_dvm *h, int mode, const FrArgs &A) {
    switch (h->p) {
        case 1: return launch_p<Real, SReal, 1, NMOM, ER>(h, mode, A);
        case 2: return launch_p<Real, SReal, 2, NMOM, ER>(h, mode, A);
        case 3: return launch_p<Real, SReal, 3, NMOM, ER>(h, mode, A);
    }
    return h->fail(FR_DVM_EUNSUPPORTED, "order");
}

// Streaming copy with 16-byte accesses, grid-stride, four loads in flight
// per lane before the stores.
__global__ __launch_bounds__(256) void k_copy16(uint4 *__restrict__ dst, const uint4 *__restrict__ src, int64_t n) {
    const int64_t st = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * st < n; i += 4 * st) {
        const uint4 a = src[i], b = src[i + st], c = src[i + 2 * st], d = src[i + 3 * st];
        dst[i] = a;
        dst[i + st] = b;
        dst[i + 2 * st] = c;
        dst[i + 3 * st] = d;
    }
    for (; i < n; i += st) dst[i] = src[i];
}

}  // namespace

namespace {
void fill_args(fr_dvm *h, const StageArgs &sa, int do_traces, int do_moments, FrArgs &A) {
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
    A.inv_nx = 1.0f / (float)h->vg.nv[0];
    A.inv_nxy = 1.0f / (float)(h->vg.nv[0] * h->vg.nv[1]);
    A.tl = h->tl;
    A.nu = h->vg.nu;
    A.gfac = h->d_gfac;
    A.nbr = h->d_nbr;
    A.wx3 = h->d_wx3;
    A.wrow = h->d_wrow;
    A.sa = sa;
    A.do_traces = do_traces;
    A.do_moments = do_moments;
    A.elem_comp = h->tl.elem / h->ncomp;
    A.gfp = h->d_gfp;
}
}  // namespace

int launch_fr_axis(fr_dvm *h, int mode, const StageArgs &sa, int do_traces, int do_moments) {
    if (sa.ecount < 0 || sa.e0 < 0 || (sa.ecount ? sa.e0 + sa.ecount > h->ne : sa.e0 != 0))
        return h->fail(FR_DVM_EINVAL, "element range");
    FrArgs A;
    fill_args(h, sa, do_traces, do_moments, A);
    if (h->prm.precision == FR_DVM_FP32_DEV && mode == MODE_STAGE && (sa.in_dev || sa.out_dev)) {
        // FP32 arithmetic on deviations from element references (monatomic)
        if (!sa.ref_prev || !sa.ref_cur) return h->fail(FR_DVM_EINVAL, "element references missing");
        if (h->nmom == 5) return launch_np<float, float, 5, true>(h, mode, A);
        if (h->nmom == 10) return launch_np<float, float, 10, true>(h, mode, A);
        return h->fail(FR_DVM_EUNSUPPORTED, "FP32 deviation storage needs a monatomic gas");
    }
    const bool fp64 = h->prm.precision == FR_DVM_FP64;
    switch (h->nmom) {
        case 5: return fp64 ? launch_np<double, double, 5>(h, mode, A) : launch_np<float, float, 5>(h, mode, A);
        case 6: return fp64 ? launch_np<double, double, 6>(h, mode, A) : launch_np<float, float, 6>(h, mode, A);
        case 10: return fp64 ? launch_np<double, double, 10>(h, mode, A) : launch_np<float, float, 10>(h, mode, A);
    }
    return fp64 ? launch_np<double, double, 11>(h, mode, A) : launch_np<float, float, 11>(h, mode, A);
}

int launch_elem_ref(fr_dvm *h, double *ref) {
    StageArgs sa;
    std::memset(&sa, 0, sizeof(sa));
    sa.eq = h->d_eq;
    FrArgs A;
    fill_args(h, sa, 0, 0, A);
    if (h->nmom == 5)
        hipLaunchKernelGGL(k_elem_ref<5>, dim3((unsigned)h->ne), dim3(kRefBlock), 0, h->stream, A, h->ns, ref);
    else if (h->nmom == 10)
        hipLaunchKernelGGL(k_elem_ref<10>, dim3((unsigned)h->ne), dim3(kRefBlock), 0, h->stream, A, h->ns, ref);
    else
        return h->fail(FR_DVM_EUNSUPPORTED, "FP32 deviation storage needs a monatomic gas");
    hipError_t st = hipGetLastError();
    if (st != hipSuccess) return h->fail(FR_DVM_EHIP, std::string("reference kernel launch: ") + hipGetErrorString(st));
    return FR_DVM_OK;
}

}  // namespace frdvm

extern "C" int fr_dvm_hbm_copy(void *dst, const void *src, size_t nbytes, void *stream) {
    if (!dst || !src || nbytes % 16 != 0) return FR_DVM_EINVAL;
    const char *d = static_cast<const char *>(dst), *s = static_cast<const char *>(src);
    if (d < s + nbytes && s < d + nbytes) return FR_DVM_EINVAL;
    int64_t n = (int64_t)(nbytes / 16);
    if (n == 0) return FR_DVM_OK;
    int64_t blocks = (n + 1023) / 1024;
    if (blocks > 256 * 32) blocks = 256 * 32;
    hipLaunchKernelGGL(frdvm::k_copy16, dim3((unsigned)blocks), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                       static_cast<uint4 *>(dst), static_cast<const uint4 *>(src), n);
    return hipGetLastError() == hipSuccess ? FR_DVM_OK : FR_DVM_EHIP;
}
