// Scoring network of the learned reduction policy (gfx950).
//
// A fully connected network in fp32: 16 inputs -> 128 -> 128 -> 1 with ReLU
// after both hidden layers.  Parameters are one flat vector:
//   W1[16][128], b1[128], W2[128][128], b2[128], w3[128], b3
// (row-major, W[k][j] multiplies input k into unit j).  Training minimises
// the mean squared error (1/R) sum_r (y_r - t_r)^2 with Adam.
//
// Each workgroup takes 64 rows.  The hidden activations of its rows and W2
// (rows padded to 129 floats so that both W2[k][.] and W2[.][j] sweeps are
// free of bank conflicts) sit in LDS; the gradient kernel writes one partial
// gradient per workgroup and a second kernel sums the partials in a fixed
// order, so a gradient is reproducible bit for bit.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace crf {

constexpr int kIn = 16, kHid = 128;
constexpr int kOW1 = 0, kOB1 = kIn * kHid, kOW2 = kOB1 + kHid, kOB2 = kOW2 + kHid * kHid, kOW3 = kOB2 + kHid,
              kOB3 = kOW3 + kHid, kNParam = kOB3 + 1;
constexpr int kRowsWG = 64, kThr = 256, kW2S = kHid + 1;

constexpr size_t mlp_lds_bytes() {
    return sizeof(float) * ((size_t)kHid * kW2S + 2 * (size_t)kRowsWG * kHid + (size_t)kRowsWG * kIn + 2 * kRowsWG);
}

struct MlpLds {
    float *W2s, *H1, *H2, *Xs, *ys, *dy;
};

__device__ static MlpLds mlp_lds(unsigned char *lds) {
    MlpLds L;
    L.W2s = reinterpret_cast<float *>(lds);
    L.H1 = L.W2s + kHid * kW2S;
    L.H2 = L.H1 + kRowsWG * kHid;
    L.Xs = L.H2 + kRowsWG * kHid;
    L.ys = L.Xs + kRowsWG * kIn;
    L.dy = L.ys + kRowsWG;
    return L;
}

// Forward pass of rows [r0, r0 + 64) (rows >= R are zero inputs).
__device__ static void mlp_forward_block(const float *__restrict__ W, const float *__restrict__ X, int R, int r0,
                                         const MlpLds &L) {
    const int tid = threadIdx.x;
    for (int idx = tid; idx < kHid * kHid; idx += kThr) L.W2s[(idx / kHid) * kW2S + idx % kHid] = W[kOW2 + idx];
    for (int idx = tid; idx < kRowsWG * kIn; idx += kThr) {
        const int r = r0 + idx / kIn;
        L.Xs[idx] = r < R ? X[(size_t)r * kIn + idx % kIn] : 0.f;
    }
    __syncthreads();
    for (int idx = tid; idx < kRowsWG * kHid; idx += kThr) {
        const int r = idx / kHid, j = idx % kHid;
        float a = W[kOB1 + j];
#pragma unroll
        for (int k = 0; k < kIn; k++) a = fmaf(L.Xs[r * kIn + k], W[kOW1 + k * kHid + j], a);
        L.H1[idx] = fmaxf(a, 0.f);
    }
    __syncthreads();
    for (int idx = tid; idx < kRowsWG * kHid; idx += kThr) {
        const int r = idx / kHid, j = idx % kHid;
        float a = W[kOB2 + j];
        for (int k = 0; k < kHid; k++) a = fmaf(L.H1[r * kHid + k], L.W2s[k * kW2S + j], a);
        L.H2[idx] = fmaxf(a, 0.f);
    }
    __syncthreads();
    if (tid < kRowsWG) {
        float a = W[kOB3];
        for (int j = 0; j < kHid; j++) a = fmaf(L.H2[tid * kHid + j], W[kOW3 + j], a);
        L.ys[tid] = a;
    }
    __syncthreads();
}

__global__ __launch_bounds__(kThr) void k_mlp_forward(const float *__restrict__ W, const float *__restrict__ X, int R,
                                                      float *__restrict__ Y) {
    extern __shared__ __align__(16) unsigned char lds[];
    const MlpLds L = mlp_lds(lds);
    const int r0 = blockIdx.x * kRowsWG;
    mlp_forward_block(W, X, R, r0, L);
    if (threadIdx.x < kRowsWG && r0 + (int)threadIdx.x < R) Y[r0 + threadIdx.x] = L.ys[threadIdx.x];
}

// Partial gradient of (1/R) sum (y - t)^2 over this workgroup's rows, and its
// partial loss, into part[blockIdx.x][0 .. kNParam].
__global__ __launch_bounds__(kThr) void k_mlp_grad(const float *__restrict__ W, const float *__restrict__ X,
                                                   const float *__restrict__ T, int R, float *__restrict__ part) {
    extern __shared__ __align__(16) unsigned char lds[];
    const MlpLds L = mlp_lds(lds);
    const int tid = threadIdx.x, r0 = blockIdx.x * kRowsWG;
    mlp_forward_block(W, X, R, r0, L);
    float *G = part + (size_t)blockIdx.x * (kNParam + 1);
    if (tid < kRowsWG) {
        const bool ok = r0 + tid < R;
        const float e = ok ? L.ys[tid] - T[r0 + tid] : 0.f;
        L.dy[tid] = 2.f * e / (float)R;
        L.ys[tid] = e * e;  // squared error, summed below
    }
    __syncthreads();
    if (tid == 0) {
        float s = 0.f, sd = 0.f;
        for (int r = 0; r < kRowsWG; r++) {
            s += L.ys[r];
            sd += L.dy[r];
        }
        G[kNParam] = s / (float)R;
        G[kOB3] = sd;
    }
    // w3 and the output-layer delta dH2 = dy w3 [H2 > 0] (in place of H2)
    if (tid < kHid) {
        float a = 0.f;
        for (int r = 0; r < kRowsWG; r++) a = fmaf(L.H2[r * kHid + tid], L.dy[r], a);
        G[kOW3 + tid] = a;
    }
    __syncthreads();
    for (int idx = tid; idx < kRowsWG * kHid; idx += kThr) {
        const int r = idx / kHid, j = idx % kHid;
        L.H2[idx] = L.H2[idx] > 0.f ? L.dy[r] * W[kOW3 + j] : 0.f;
    }
    __syncthreads();
    // W2, b2
    for (int idx = tid; idx < kHid * kHid; idx += kThr) {
        const int k = idx / kHid, j = idx % kHid;
        float a = 0.f;
        for (int r = 0; r < kRowsWG; r++) a = fmaf(L.H1[r * kHid + k], L.H2[r * kHid + j], a);
        G[kOW2 + idx] = a;
    }
    if (tid < kHid) {
        float a = 0.f;
        for (int r = 0; r < kRowsWG; r++) a += L.H2[r * kHid + tid];
        G[kOB2 + tid] = a;
    }
    __syncthreads();
    // dH1 = (dH2 W2^T) [H1 > 0] (in place of H1: each entry reads only its own H1)
    for (int idx = tid; idx < kRowsWG * kHid; idx += kThr) {
        const int r = idx / kHid, k = idx % kHid;
        float a = 0.f;
        for (int j = 0; j < kHid; j++) a = fmaf(L.H2[r * kHid + j], L.W2s[k * kW2S + j], a);
        L.H1[idx] = L.H1[idx] > 0.f ? a : 0.f;
    }
    __syncthreads();
    // W1, b1
    for (int idx = tid; idx < kIn * kHid; idx += kThr) {
        const int i = idx / kHid, k = idx % kHid;
        float a = 0.f;
        for (int r = 0; r < kRowsWG; r++) a = fmaf(L.Xs[r * kIn + i], L.H1[r * kHid + k], a);
        G[kOW1 + idx] = a;
    }
    if (tid < kHid) {
        float a = 0.f;
        for (int r = 0; r < kRowsWG; r++) a += L.H1[r * kHid + tid];
        G[kOB1 + tid] = a;
    }
}

// grad[i] = sum_b part[b][i] in the order b = 0, 1, ...
__global__ __launch_bounds__(kThr) void k_mlp_reduce(const float *__restrict__ part, int nparts,
                                                     float *__restrict__ grad) {
    const int i = blockIdx.x * kThr + threadIdx.x;
    if (i > kNParam) return;
    float a = 0.f;
    for (int b = 0; b < nparts; b++) a += part[(size_t)b * (kNParam + 1) + i];
    grad[i] = a;
}

// Adam (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// w -= lr (m / c1) / (sqrt(v / c2) + eps) with c1 = 1 - b1^t, c2 = 1 - b2^t.
__global__ __launch_bounds__(kThr) void k_adam(float *__restrict__ W, float *__restrict__ m, float *__restrict__ v,
                                               const float *__restrict__ g, float lr, float b1, float b2, float eps,
                                               float c1, float c2) {
    const int i = blockIdx.x * kThr + threadIdx.x;
    if (i >= kNParam) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    W[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

int mlp_param_count() { return kNParam; }

static hipError_t set_lds(const void *fn) {
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)mlp_lds_bytes());
}

hipError_t launch_mlp_forward(const float *W, const float *X, int R, float *Y, hipStream_t stream) {
    if (R <= 0) return hipSuccess;
    hipError_t e = set_lds((const void *)k_mlp_forward);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_forward, dim3((R + kRowsWG - 1) / kRowsWG), dim3(kThr), mlp_lds_bytes(), stream, W, X, R,
                       Y);
    return hipGetLastError();
}

// part needs ceil(R / 64) * (kNParam + 1) floats; grad kNParam + 1 (the last is the loss).
hipError_t launch_mlp_grad(const float *W, const float *X, const float *T, int R, float *part, float *grad,
                           hipStream_t stream) {
    if (R <= 0) return hipErrorInvalidValue;
    hipError_t e = set_lds((const void *)k_mlp_grad);
    if (e != hipSuccess) return e;
    const int nb = (R + kRowsWG - 1) / kRowsWG;
    hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(kThr), mlp_lds_bytes(), stream, W, X, T, R, part);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kNParam + 1 + kThr - 1) / kThr), dim3(kThr), 0, stream, part, nb, grad);
    return hipGetLastError();
}

hipError_t launch_adam(float *W, float *m, float *v, const float *g, float lr, float b1, float b2, float eps, float c1,
                       float c2, hipStream_t stream) {
    hipLaunchKernelGGL(k_adam, dim3((kNParam + kThr - 1) / kThr), dim3(kThr), 0, stream, W, m, v, g, lr, b1, b2, eps,
                       c1, c2);
    return hipGetLastError();
}

}  // namespace crf
