// Training and inference kernels of the learned Newton initial guess
// (include/fr_dvm_mlp.h), FP32 on gfx950.
//
// The dense layers are small GEMMs (batch x 64 x 64) run on the matrix cores
// with v_mfma_f32_16x16x4_f32: one wave per 16x16 output tile, K stepped by 4.
// Bias/activation, loss, column sums and Adam are plain elementwise kernels.
// Every reduction has a fixed order, so training is bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "../../include/fr_dvm_mlp.h"
#include "frdvm_common.h"

namespace frdvm {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// C[M][N] = sum_k A(m,k) B(k,n);  A(m,k) = tA ? A[k lda + m] : A[m lda + k],
// B(k,n) = tB ? B[n ldb + k] : B[k ldb + n].  Operand layout of the 16x16x4
// FP32 MFMA: lane l supplies A[l%16][l/16] and B[l/16][l%16] and receives
// D[4 (l/16) + i][l%16], i = 0..3.
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const float *__restrict__ A, int lda, int tA,
                                              const float *__restrict__ B, int ldb, int tB, float *__restrict__ C,
                                              int ldc) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tilesN = (N + 15) / 16;
    const int tile = blockIdx.x * 4 + wave;
    const int tm = tile / tilesN, tn = tile % tilesN;
    if (tm * 16 >= M) return;  // whole wave leaves together
    const int r16 = lane & 15, q = lane >> 4;
    const int m = tm * 16 + r16, n = tn * 16 + r16;
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 4) {
        const int k = k0 + q;
        float a = 0.f, b = 0.f;
        if (m < M && k < K) a = tA ? A[(int64_t)k * lda + m] : A[(int64_t)m * lda + k];
        if (n < N && k < K) b = tB ? B[(int64_t)n * ldb + k] : B[(int64_t)k * ldb + n];
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int mm = tm * 16 + 4 * q + i, nn = tn * 16 + r16;
        if (mm < M && nn < N) C[(int64_t)mm * ldc + nn] = acc[i];
    }
}

__device__ __forceinline__ float silu(float x) { return x / (1.f + __expf(-x)); }
__device__ __forceinline__ float dsilu(float x) {
    float s = 1.f / (1.f + __expf(-x));
    return s * (1.f + x * (1.f - s));
}

// Z += bias (per column); A = silu(Z) when act, else nothing.
__global__ void k_bias_act(int64_t M, int N, float *Z, const float *bias, float *A, int act) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M * N) return;
    float z = Z[i] + bias[i % N];
    Z[i] = z;
    if (act) A[i] = silu(z);
}

// delta = (Y - T)/B in place of Y; per-block partial sums of |Y - T|^2 / (2B).
__global__ __launch_bounds__(256) void k_loss_delta(int64_t B, float *Y, const float *T, float *partial) {
    __shared__ float red[256];
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float l = 0.f;
    if (i < B * 5) {
        float r = Y[i] - T[i];
        l = 0.5f * r * r / (float)B;
        Y[i] = r / (float)B;
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_sum(int n, const float *partial, float *out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        float s = 0.f;
        for (int i = 0; i < n; ++i) s += partial[i];
        out[0] = s;
    }
}

__global__ void k_dsilu_mul(int64_t n, float *D, const float *Z) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) D[i] *= dsilu(Z[i]);
}

// out[n] = sum over rows of D[m][n] (sequential per column: fixed order).
__global__ void k_colsum(int64_t M, int N, const float *D, float *out) {
    int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int64_t m = 0; m < M; ++m) s += D[m * N + n];
    out[n] = s;
}

__global__ void k_adam(int64_t n, float *w, const float *g, float *m, float *v, float c1, float c2, float lr) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float mi = 0.9f * m[i] + 0.1f * g[i];
    float vi = 0.999f * v[i] + 0.001f * g[i] * g[i];
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

__global__ void k_affine(int64_t B, const float *Y, const float *scale, const float *offset, float *out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < B * 5) out[i] = Y[i] * scale[i % 5] + offset[i % 5];
}

struct Layout {
    size_t W[4], b[4], scale, offset, total;
    int in[4], out[4];
};

Layout layout(int H) {
    Layout L;
    int ins[4] = {FR_MLP_INPUTS, H, H, H}, outs[4] = {H, H, H, 5};
    size_t o = 0;
    for (int l = 0; l < 4; ++l) {
        L.in[l] = ins[l];
        L.out[l] = outs[l];
        L.W[l] = o;
        o += (size_t)outs[l] * ins[l];
        L.b[l] = o;
        o += outs[l];
    }
    L.scale = o;
    L.offset = o + 5;
    L.total = o + 10;
    return L;
}

struct Work {
    float *Z[3], *A[3], *Y, *Da, *Db, *partial;
};

Work carve(float *work, int H, int64_t B) {
    Work w;
    size_t bh = (size_t)B * H;
    for (int l = 0; l < 3; ++l) {
        w.Z[l] = work + (2 * l) * bh;
        w.A[l] = work + (2 * l + 1) * bh;
    }
    w.Y = work + 6 * bh;
    w.Da = w.Y + (size_t)B * 5;
    w.Db = w.Da + bh;
    w.partial = w.Db + bh;
    return w;
}

void gemm(hipStream_t s, int M, int N, int K, const float *A, int lda, int tA, const float *B, int ldb, int tB,
          float *C, int ldc) {
    int tiles = ((M + 15) / 16) * ((N + 15) / 16);
    hipLaunchKernelGGL(k_gemm, dim3((tiles + 3) / 4), dim3(256), 0, s, M, N, K, A, lda, tA, B, ldb, tB, C, ldc);
}

unsigned blocks(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// Forward pass into the workspace; Y holds the normalised output.
void forward(hipStream_t s, int H, const float *w, const float *X, int64_t B, const Work &wk) {
    Layout L = layout(H);
    const float *a = X;
    for (int l = 0; l < 3; ++l) {
        gemm(s, (int)B, H, L.in[l], a, L.in[l], 0, w + L.W[l], L.in[l], 1, wk.Z[l], H);
        hipLaunchKernelGGL(k_bias_act, dim3(blocks(B * H)), dim3(256), 0, s, B, H, wk.Z[l], w + L.b[l], wk.A[l], 1);
        a = wk.A[l];
    }
    gemm(s, (int)B, 5, H, a, H, 0, w + L.W[3], H, 1, wk.Y, 5);
    hipLaunchKernelGGL(k_bias_act, dim3(blocks(B * 5)), dim3(256), 0, s, B, 5, wk.Y, w + L.b[3], (float *)nullptr, 0);
}

// Scratch of fr_mlp_forward_noalloc: two [B][H] activation buffers used in
// turn (each layer's GEMM writes one from the other, bias and SiLU in place)
// and the [B][5] output.  In host code `scratch` names a host-side stand-in;
// kernels receive the device address from hipGetSymbolAddress, kept per GPU.
static __device__ __align__(256) float scratch[FR_MLP_NOALLOC_FLOATS];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
float *scratch_dev[kMaxDevices] = {};

// Device address of the current GPU's scratch, looked up once per GPU with
// that GPU current.
int scratch_ptr(float **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return FR_DVM_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return FR_DVM_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return FR_DVM_EHIP;
        scratch_dev[dev] = static_cast<float *>(ptr);
    }
    *out = scratch_dev[dev];
    return FR_DVM_OK;
}

int hip_ok(const char *what) {
    (void)what;
    return hipGetLastError() == hipSuccess ? FR_DVM_OK : FR_DVM_EHIP;
}

}  // namespace
}  // namespace frdvm

using namespace frdvm;

extern "C" size_t fr_mlp_param_count(int H) { return H > 0 ? layout(H).total : 0; }

extern "C" size_t fr_mlp_workspace_floats(int H, int64_t B) {
    return (size_t)8 * B * H + (size_t)5 * B + ((size_t)B * 5 + 255) / 256 + 16;
}

extern "C" int fr_mlp_forward(int H, const float *w, const float *X, int64_t B, float *dz, float *work, void *stream) {
    if (H < 1 || H > 1024 || B < 0 || !w || !work || (B > 0 && (!X || !dz))) return FR_DVM_EINVAL;
    if (B == 0) return FR_DVM_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Work wk = carve(work, H, B);
    forward(s, H, w, X, B, wk);
    Layout L = layout(H);
    hipLaunchKernelGGL(k_affine, dim3(blocks(B * 5)), dim3(256), 0, s, B, wk.Y, w + L.scale, w + L.offset, dz);
    return hip_ok("mlp forward");
}

extern "C" int fr_mlp_forward_noalloc(int H, const float *w, const float *X, int64_t B, float *dz, void *stream) {
    if (H < 1 || H > 1024 || B < 0 || !w || (B > 0 && (!X || !dz))) return FR_DVM_EINVAL;
    if (B == 0) return FR_DVM_OK;
    if ((size_t)B > FR_MLP_NOALLOC_FLOATS / (size_t)(2 * H + 5)) return FR_DVM_ESCRATCH;
    float *base = nullptr;
    int rc = scratch_ptr(&base);
    if (rc) return rc;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Layout L = layout(H);
    float *act[2] = {base, base + (size_t)B * H};
    float *Y = base + (size_t)2 * B * H;
    const float *a = X;
    for (int l = 0; l < 3; ++l) {
        float *z = act[l & 1];
        gemm(s, (int)B, H, L.in[l], a, L.in[l], 0, w + L.W[l], L.in[l], 1, z, H);
        hipLaunchKernelGGL(k_bias_act, dim3(blocks(B * H)), dim3(256), 0, s, B, H, z, w + L.b[l], z, 1);
        a = z;
    }
    gemm(s, (int)B, 5, H, a, H, 0, w + L.W[3], H, 1, Y, 5);
    hipLaunchKernelGGL(k_bias_act, dim3(blocks(B * 5)), dim3(256), 0, s, B, 5, Y, w + L.b[3], (float *)nullptr, 0);
    hipLaunchKernelGGL(k_affine, dim3(blocks(B * 5)), dim3(256), 0, s, B, Y, w + L.scale, w + L.offset, dz);
    return hip_ok("mlp forward (no allocation)");
}

extern "C" int fr_mlp_grad(int H, const float *w, const float *X, const float *T, int64_t B, float *grad, float *loss,
                           float *work, void *stream) {
    if (H < 1 || H > 1024 || B < 1 || !w || !X || !T || !grad || !loss || !work) return FR_DVM_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Layout L = layout(H);
    Work wk = carve(work, H, B);
    forward(s, H, w, X, B, wk);
    const unsigned nb = blocks(B * 5);
    hipLaunchKernelGGL(k_loss_delta, dim3(nb), dim3(256), 0, s, B, wk.Y, T, wk.partial);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(64), 0, s, (int)nb, wk.partial, loss);
    // output layer: delta in Y [B][5]
    const float *delta = wk.Y;
    int dn = 5;
    float *bufs[2] = {wk.Da, wk.Db};
    for (int l = 3; l >= 0; --l) {
        const float *ain = l == 0 ? X : wk.A[l - 1];
        const int nin = L.in[l];
        // dW_l = delta^T a_in  (out x in), db_l = column sums of delta
        gemm(s, dn, nin, (int)B, delta, dn, 1, ain, nin, 0, grad + L.W[l], nin);
        hipLaunchKernelGGL(k_colsum, dim3(blocks(dn, 64)), dim3(64), 0, s, B, dn, delta, grad + L.b[l]);
        if (l == 0) break;
        // delta_{l-1} = (delta W_l) * silu'(Z_{l-1})
        float *nd = bufs[l & 1];
        gemm(s, (int)B, nin, dn, delta, dn, 0, w + L.W[l], nin, 0, nd, nin);
        hipLaunchKernelGGL(k_dsilu_mul, dim3(blocks(B * nin)), dim3(256), 0, s, B * nin, nd, wk.Z[l - 1]);
        delta = nd;
        dn = nin;
    }
    (void)hipMemsetAsync(grad + L.scale, 0, 10 * sizeof(float), s);
    return hip_ok("mlp grad");
}

extern "C" int fr_mlp_adam(int H, float *w, const float *grad, float *m, float *v, int step, float lr, void *stream) {
    if (H < 1 || !w || !grad || !m || !v || step < 1) return FR_DVM_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int64_t n = (int64_t)layout(H).scale;  // network weights only
    float c1 = 1.f - powf(0.9f, (float)step), c2 = 1.f - powf(0.999f, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(blocks(n)), dim3(256), 0, s, n, w, grad, m, v, c1, c2, lr);
    return hip_ok("adam");
}
