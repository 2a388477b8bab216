// FP64 vector kernels of the Krylov solver: fused multi-dot products,
// orthogonalisation updates, norms and multi-axpys (Sec. 4.1 of the paper
// uses FGMRES; these are its orthogonalisation and update steps).
//
// Reductions are deterministic: every launch uses the same grid of
// RED_BLOCKS x RED_THREADS threads with a grid-stride loop, each block reduces
// its threads in a fixed LDS tree, and one block adds the block partials in a
// fixed order.  Results therefore do not depend on timing or on other work
// sharing the device.
#include "kernels.h"

namespace iim {

constexpr int KCH = 12;  // vectors handled per pass (registers per thread)

__device__ inline void block_reduce_store(double* vals, int k, double* part, int partial_stride) {
    __shared__ double sh[RED_THREADS];
    for (int i = 0; i < k; ++i) {
        sh[threadIdx.x] = vals[i];
        __syncthreads();
        for (int off = RED_THREADS / 2; off > 0; off >>= 1) {
            if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[(int64_t)i * partial_stride + blockIdx.x] = sh[0];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(RED_THREADS) k_final(const double* part, int k, double* out, int mode) {
    __shared__ double sh[RED_THREADS];
    for (int i = 0; i < k; ++i) {
        double v = 0.0;
        for (int b = threadIdx.x; b < RED_BLOCKS; b += RED_THREADS) {
            double p = part[(int64_t)i * RED_BLOCKS + b];
            v = mode == 1 ? fmax(v, p) : v + p;
        }
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int off = RED_THREADS / 2; off > 0; off >>= 1) {
            if (threadIdx.x < off)
                sh[threadIdx.x] = mode == 1 ? fmax(sh[threadIdx.x], sh[threadIdx.x + off])
                                            : sh[threadIdx.x] + sh[threadIdx.x + off];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            out[i] = sh[0];
            if (mode == 1) out[1] = sh[0] > 0.0 ? 1.0 / sh[0] : 1.0;
        }
        __syncthreads();
    }
}

static void final_sum(const double* part, int k, double* out, hipStream_t s, int mode = 0) {
    hipLaunchKernelGGL(k_final, dim3(1), dim3(RED_THREADS), 0, s, part, k, out, mode);
    IIM_LAUNCH_CHECK();
}

__global__ void __launch_bounds__(RED_THREADS) k_multidot(const double* V, int64_t ld, int k0, int k,
                                                          const double* w, int64_t n, double* part) {
    double acc[KCH];
#pragma unroll
    for (int i = 0; i < KCH; ++i) acc[i] = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        double we = w[e];
#pragma unroll
        for (int i = 0; i < KCH; ++i)
            if (i < k) acc[i] += V[(int64_t)(k0 + i) * ld + e] * we;
    }
    block_reduce_store(acc, k, part + (int64_t)k0 * RED_BLOCKS, RED_BLOCKS);
}

void run_multidot(const double* V, int64_t ld, int k, const double* w, int64_t n, double* part, double* out,
                  hipStream_t s) {
    for (int k0 = 0; k0 < k; k0 += KCH) {
        int kk = std::min(KCH, k - k0);
        hipLaunchKernelGGL(k_multidot, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, V, ld, k0, kk, w, n, part);
        IIM_LAUNCH_CHECK();
    }
    final_sum(part, k, out, s);
}

// w -= sum_i h_i V_i (all k at once), then dots of the updated w
__global__ void __launch_bounds__(RED_THREADS) k_update_dot(const double* V, int64_t ld, int k, const double* h,
                                                            double* w, int64_t n, int k2, int with_norm,
                                                            double* part) {
    double acc[KCH + 1];
#pragma unroll
    for (int i = 0; i <= KCH; ++i) acc[i] = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        double we = w[e];
        for (int i = 0; i < k; ++i) we -= h[i] * V[(int64_t)i * ld + e];
        w[e] = we;
#pragma unroll
        for (int i = 0; i < KCH; ++i)
            if (i < k2) acc[i] += V[(int64_t)i * ld + e] * we;
        acc[KCH] += we * we;
    }
    if (with_norm) acc[k2] = acc[KCH];
    block_reduce_store(acc, k2 + (with_norm ? 1 : 0), part, RED_BLOCKS);
}

void run_update_dot(const double* V, int64_t ld, int k, const double* h, double* w, int64_t n, int k2,
                    int with_norm, double* part, double* out, hipStream_t s) {
    if (k2 > KCH) throw Error(IIM_E_INVALID_ARG, "update_dot: too many vectors");
    hipLaunchKernelGGL(k_update_dot, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, V, ld, k, h, w, n, k2, with_norm,
                       part);
    IIM_LAUNCH_CHECK();
    final_sum(part, k2 + (with_norm ? 1 : 0), out, s);
}

__global__ void k_normalize(const double* x, const double* nrm2, double* y, int64_t n) {
    double inv = 1.0 / sqrt(*nrm2);
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        y[e] = x[e] * inv;
}

void run_normalize(const double* x, const double* nrm2, double* y, int64_t n, hipStream_t s) {
    int blocks = (int)std::min<int64_t>(cdiv(n, 256), 4096);
    hipLaunchKernelGGL(k_normalize, dim3(blocks), dim3(256), 0, s, x, nrm2, y, n);
    IIM_LAUNCH_CHECK();
}

__global__ void k_axpy_multi(const double* Z, int64_t ld, int k, const double* y, double* x, int64_t n) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        double v = x[e];
        for (int i = 0; i < k; ++i) v += y[i] * Z[(int64_t)i * ld + e];
        x[e] = v;
    }
}

void run_axpy_multi(const double* Z, int64_t ld, int k, const double* y, double* x, int64_t n, hipStream_t s) {
    if (k == 0) return;
    int blocks = (int)std::min<int64_t>(cdiv(n, 256), 4096);
    hipLaunchKernelGGL(k_axpy_multi, dim3(blocks), dim3(256), 0, s, Z, ld, k, y, x, n);
    IIM_LAUNCH_CHECK();
}

__global__ void k_axpby(double a, const double* x, double b, double* y, int64_t n) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        y[e] = a * x[e] + b * y[e];
}

void run_axpby(double a, const double* x, double b, double* y, int64_t n, hipStream_t s) {
    int blocks = (int)std::min<int64_t>(cdiv(n, 256), 4096);
    hipLaunchKernelGGL(k_axpby, dim3(blocks), dim3(256), 0, s, a, x, b, y, n);
    IIM_LAUNCH_CHECK();
}

void run_copy(const double* x, double* y, int64_t n, hipStream_t s) {
    IIM_HIP(hipMemcpyAsync(y, x, n * sizeof(double), hipMemcpyDeviceToDevice, s));
}

__global__ void __launch_bounds__(RED_THREADS) k_absmax(const double* x, int64_t n, double* part) {
    __shared__ double sh[RED_THREADS];
    double v = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        v = fmax(v, fabs(x[e]));
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = RED_THREADS / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

void run_absmax(const double* x, int64_t n, double* part, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_absmax, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, x, n, part);
    IIM_LAUNCH_CHECK();
    final_sum(part, 1, out, s, 1);
}

__global__ void __launch_bounds__(RED_THREADS) k_norm2(const double* x, int64_t n, double* part) {
    double acc[1] = {0.0};
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        acc[0] += x[e] * x[e];
    block_reduce_store(acc, 1, part, RED_BLOCKS);
}

void run_norm2(const double* x, int64_t n, double* part, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_norm2, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, x, n, part);
    IIM_LAUNCH_CHECK();
    final_sum(part, 1, out, s);
}

}  // namespace iim
