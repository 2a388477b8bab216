// FP64 vector kernels of the Krylov solver: fused multi-dot products,
// orthogonalisation updates, norms and multi-axpys (Sec. 4.1 of the paper
// uses FGMRES; these are its orthogonalisation and update steps).
//
// Every kernel streams its vectors with 16-byte (double2) loads: vectors start
// on 16-byte boundaries (basis vectors sit at an even leading dimension) and an
// odd trailing element is handled by one thread.
//
// Reductions are deterministic: every launch uses the same grid of
// RED_BLOCKS x RED_THREADS threads with a grid-stride loop; a block reduces
// each wavefront by a fixed xor-shuffle butterfly (lane 0's value is used) and
// adds its RED_THREADS / 64 wavefront sums in order; a one-block second stage
// adds the block partials in a fixed order.  Results therefore do not depend
// on timing or on other work sharing the device.
#include "kernels.h"

namespace iim {

constexpr int KCH = 12;  // vectors handled per pass (registers per thread)
constexpr int WAVES = RED_THREADS / 64;

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// part[i * RED_BLOCKS + blockIdx.x] = block sum (mode 1: max) of vals[i], i < k
template <int K>
__device__ inline void block_reduce_store(const double (&vals)[K], int k, double* part, int mode) {
    __shared__ double sh[WAVES][K];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        if (i < k) {
            double v = mode == 1 ? wave_max_valu(vals[i]) : wave_sum_valu(vals[i]);
            if (lane == 0) sh[wv][i] = v;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < k) {
        double s = sh[0][threadIdx.x];
        for (int q = 1; q < WAVES; ++q) s = mode == 1 ? fmax(s, sh[q][threadIdx.x]) : s + sh[q][threadIdx.x];
        part[(int64_t)threadIdx.x * RED_BLOCKS + blockIdx.x] = s;
    }
}

// Second stage, one block of RED_BLOCKS threads: thread t loads partial t of
// every value at once, wavefronts reduce on the VALU, the RED_BLOCKS / 64
// wavefront results are added in order.  out[i] = sum (mode 1: max) of the
// partials of value i; mode 1 also writes out[1] = 1 / max (1 if zero).  A
// separate launch rather than a last-block-done epilogue: the epilogue's
// device-scope fences cost more than a launch on a device whose XCDs have
// separate L2 caches.
constexpr int FIN_WAVES = RED_BLOCKS / 64;

// Whether a classical Gram-Schmidt step needs its second pass.  g[0..k-1] =
// V^T w and g[k] = |w|^2 from the first pass; with rho^2 = |w|^2 - |V^T w|^2
// the norm left after one pass, the first pass alone leaves the new basis
// vector orthogonal to about eps |w| / rho and the Pythagorean norm accurate to
// about eps |w|^2 / rho^2.  The second pass is taken when rho < 1e-2 |w|,
// which bounds these by about 2e-14 and 2e-12 (a NaN also takes it, and then
// reaches the solver as a breakdown).  Every caller evaluates the same sum in
// the same order, so all blocks and the second stage agree.
constexpr double CGS_REFINE_TAU2 = 1e-4;

__device__ inline bool cgs_refine(const double* g, int k) {
    double ss = 0.0;
    for (int i = 0; i < k; ++i) ss += g[i] * g[i];
    const double w2 = g[k];
    return !(w2 - ss >= CGS_REFINE_TAU2 * w2);
}

// gate (optional): the first-pass record g of a conditional second pass.  When
// cgs_refine(g, kg) is false the pass's first stage wrote nothing; this stage
// then hands the first pass on unchanged (out[0..kg] = g[0..kg]) and records a
// zero correction (host_out[0..kg-1] = 0).  host_out[63] records whether the
// pass ran (1) or not (0).
__global__ void __launch_bounds__(RED_BLOCKS) k_final(const double* part, int k, double* out, int mode,
                                                       double* host_out, const double* gate, int kg) {
    __shared__ double sh[FIN_WAVES][KCH + 1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (gate) {
        const bool refine = cgs_refine(gate, kg);
        if (host_out && threadIdx.x == 0) host_out[63] = refine ? 1.0 : 0.0;
        if (!refine) {
            if ((int)threadIdx.x <= kg) {
                out[threadIdx.x] = gate[threadIdx.x];
                if (host_out) host_out[threadIdx.x] = (int)threadIdx.x < kg ? 0.0 : gate[kg];
            }
            return;
        }
    }
    double p[KCH + 1];
#pragma unroll
    for (int i = 0; i <= KCH; ++i) p[i] = i < k ? part[(int64_t)i * RED_BLOCKS + threadIdx.x] : 0.0;
#pragma unroll
    for (int i = 0; i <= KCH; ++i)
        if (i < k) {
            const double v = mode == 1 ? wave_max_valu(p[i]) : wave_sum_valu(p[i]);
            if (lane == 0) sh[wv][i] = v;
        }
    __syncthreads();
    if ((int)threadIdx.x < k) {
        double v = sh[0][threadIdx.x];
        for (int q = 1; q < FIN_WAVES; ++q) v = mode == 1 ? fmax(v, sh[q][threadIdx.x]) : v + sh[q][threadIdx.x];
        out[threadIdx.x] = v;
        if (host_out) host_out[threadIdx.x] = v;  // pinned host copy (zero-copy)
        if (mode == 1) out[1] = v > 0.0 ? 1.0 / v : 1.0;
    }
}

static void final_sum(const double* part, int k, double* out, hipStream_t s, int mode = 0,
                      double* host_out = nullptr, const double* gate = nullptr, int kg = 0) {
    if (k < 1 || k > KCH + 1) throw Error(IIM_E_INVALID_ARG, "reduction: 1..13 values");
    hipLaunchKernelGGL(k_final, dim3(1), dim3(RED_BLOCKS), 0, s, part, k, out, mode, host_out, gate, kg);
    IIM_LAUNCH_CHECK();
}

static void check_vec(const void* p, int64_t ld) {
    if (((uintptr_t)p & 15) || (ld & 1)) throw Error(IIM_E_INTERNAL, "vector kernels need 16-byte aligned vectors");
}

__device__ inline double2 ld2(const double* base, int64_t e) { return reinterpret_cast<const double2*>(base)[e]; }
// the same as a streaming (non-temporal) load: basis vectors are read once per
// pass over more data than the caches hold (about 6 % faster passes, measured)
__device__ inline double2 ld2_stream(const double* base, int64_t e) {
    const double2* q = reinterpret_cast<const double2*>(base) + e;
    double2 r;
    r.x = __builtin_nontemporal_load(&q->x);
    r.y = __builtin_nontemporal_load(&q->y);
    return r;
}
__device__ inline void st2(double* base, int64_t e, double2 v) { reinterpret_cast<double2*>(base)[e] = v; }
// the updated vector of a pass read and written around the caches as well: it
// is larger than they are, and the next kernel reads it whole (with these the
// update passes run 2 % faster and a cfg-4 solve 1 %, measured; the dot-only
// pass keeps cached loads of w, whose lines the update pass after it reuses)
__device__ inline double2 ld2_nt(const double* base, int64_t e) { return ld2_stream(base, e); }
__device__ inline void st2_nt(double* base, int64_t e, double2 v) {
    double2* q = reinterpret_cast<double2*>(base) + e;
    __builtin_nontemporal_store(v.x, &q->x);
    __builtin_nontemporal_store(v.y, &q->y);
}

// dots of w with V_i (i < k) and, if asked, |w|^2 right after them
__global__ void __launch_bounds__(RED_THREADS) k_multidot(const double* V, int64_t ld, int k, const double* w,
                                                          int64_t n, int with_norm, double* part) {
    double acc[KCH + 1];
#pragma unroll
    for (int i = 0; i <= KCH; ++i) acc[i] = 0.0;
    const int64_t np = n >> 1;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < np; e += (int64_t)gridDim.x * blockDim.x) {
        const double2 we = ld2(w, e);
#pragma unroll
        for (int i = 0; i < KCH; ++i)
            if (i < k) {
                const double2 v = ld2_stream(V + (int64_t)i * ld, e);
                acc[i] += v.x * we.x;
                acc[i] += v.y * we.y;
            }
        acc[KCH] += we.x * we.x;
        acc[KCH] += we.y * we.y;
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        const double we = w[n - 1];
#pragma unroll
        for (int i = 0; i < KCH; ++i)
            if (i < k) acc[i] += V[(int64_t)i * ld + n - 1] * we;
        acc[KCH] += we * we;
    }
    double outv[KCH + 1];
#pragma unroll
    for (int i = 0; i <= KCH; ++i) outv[i] = (i < k) ? acc[i] : ((i == k) ? acc[KCH] : 0.0);
    block_reduce_store(outv, k + (with_norm ? 1 : 0), part, 0);
}

void run_multidot(const double* V, int64_t ld, int k, const double* w, int64_t n, double* part, double* out,
                  hipStream_t s, double* host_out, int with_norm) {
    if (k < 1 || k > KCH) throw Error(IIM_E_INVALID_ARG, "multidot: 1..12 vectors");
    check_vec(V, ld);
    check_vec(w, 0);
    hipLaunchKernelGGL(k_multidot, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, V, ld, k, w, n, with_norm, part);
    IIM_LAUNCH_CHECK();
    final_sum(part, k + (with_norm ? 1 : 0), out, s, 0, host_out);
}

// w -= sum_i h_i V_i (all k at once), then dots of the updated w with V_i (i < k2)
// and, if asked, its squared norm; each basis vector is read once
__global__ void __launch_bounds__(RED_THREADS) k_update_dot(const double* V, int64_t ld, int k, const double* h,
                                                            double* w, int64_t n, int k2, int with_norm,
                                                            double* part, int gated) {
    // a gated pass (h = the first pass's record: k dots and |w|^2) runs only
    // when that pass left too little of w (the same test in every block)
    if (gated && !cgs_refine(h, k)) return;
    double hh[KCH], acc[KCH + 1];
#pragma unroll
    for (int i = 0; i < KCH; ++i) {
        hh[i] = i < k ? h[i] : 0.0;
        acc[i] = 0.0;
    }
    acc[KCH] = 0.0;
    const int kr = k > k2 ? k : k2;
    const int64_t np = n >> 1;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < np; e += (int64_t)gridDim.x * blockDim.x) {
        double2 we = ld2_nt(w, e);
        double2 v[KCH];
#pragma unroll
        for (int i = 0; i < KCH; ++i)
            if (i < kr) v[i] = ld2_stream(V + (int64_t)i * ld, e);
#pragma unroll
        for (int i = 0; i < KCH; ++i)
            if (i < k) {
                we.x -= hh[i] * v[i].x;
                we.y -= hh[i] * v[i].y;
            }
        st2_nt(w, e, we);
#pragma unroll
        for (int i = 0; i < KCH; ++i)
            if (i < k2) {
                acc[i] += v[i].x * we.x;
                acc[i] += v[i].y * we.y;
            }
        acc[KCH] += we.x * we.x;
        acc[KCH] += we.y * we.y;
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        const int64_t e = n - 1;
        double we = w[e];
#pragma unroll
        for (int i = 0; i < KCH; ++i)
            if (i < k) we -= hh[i] * V[(int64_t)i * ld + e];
        w[e] = we;
#pragma unroll
        for (int i = 0; i < KCH; ++i)
            if (i < k2) acc[i] += V[(int64_t)i * ld + e] * we;
        acc[KCH] += we * we;
    }
    // dots in slots 0..k2-1, the norm right after them
    double outv[KCH + 1];
#pragma unroll
    for (int i = 0; i <= KCH; ++i) outv[i] = (i < k2) ? acc[i] : ((i == k2) ? acc[KCH] : 0.0);
    block_reduce_store(outv, k2 + (with_norm ? 1 : 0), part, 0);
}

void run_update_dot_stage1(const double* V, int64_t ld, int k, const double* h, double* w, int64_t n, int k2,
                           int with_norm, double* part, hipStream_t s) {
    if (k > KCH || k2 > KCH) throw Error(IIM_E_INVALID_ARG, "update_dot: too many vectors");
    check_vec(V, ld);
    check_vec(w, 0);
    hipLaunchKernelGGL(k_update_dot, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, V, ld, k, h, w, n, k2, with_norm,
                       part, 0);
    IIM_LAUNCH_CHECK();
}

void run_update_dot(const double* V, int64_t ld, int k, const double* h, double* w, int64_t n, int k2,
                    int with_norm, double* part, double* out, hipStream_t s, double* host_out, bool gated) {
    if (k > KCH || k2 > KCH) throw Error(IIM_E_INVALID_ARG, "update_dot: too many vectors");
    check_vec(V, ld);
    check_vec(w, 0);
    if (k2 + (with_norm ? 1 : 0) < 1) throw Error(IIM_E_INVALID_ARG, "update_dot: nothing to reduce");
    if (gated && (k2 != k || !with_norm)) throw Error(IIM_E_INVALID_ARG, "update_dot: a gated pass is a full CGS pass");
    hipLaunchKernelGGL(k_update_dot, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, V, ld, k, h, w, n, k2, with_norm,
                       part, gated ? 1 : 0);
    IIM_LAUNCH_CHECK();
    final_sum(part, k2 + (with_norm ? 1 : 0), out, s, 0, host_out, gated ? h : nullptr, k);
}

// Last classical Gram-Schmidt update fused with the normalisation:
//   y = (w - sum_i h_i V_i) / sqrt(nrm2),  nrm2 = h[k] - sum_i h_i^2,
// where h[0..k-1] = V^T w and h[k] = |w|^2 come from the pass that read w.  With
// V orthonormal, |w - V h|^2 = |w|^2 - |h|^2 (Pythagoras).  After a first
// update h is a rounding-level correction and the difference does not cancel;
// as the only update it is used only when |h|^2 <= (1 - 1e-4) |w|^2 (see
// cgs_refine), so at most four decimal digits cancel.  nrm2 is
// floored at 0 (then y is not finite and the solver takes it as a breakdown)
// and written to *nrm2_out; block maxima of |y| over its first n_max entries
// go to part (the V-cycle's scaling of y is then one second-stage launch
// away; a bordered vector's last entry, alpha, is not an input of the cycle
// and stays out of its scale).
__global__ void __launch_bounds__(RED_THREADS) k_update_scale(const double* V, int64_t ld, int k, const double* h,
                                                              const double* w, double* y, int64_t n, int64_t n_max,
                                                              double* nrm2_out, double* nrm2_host, double* part) {
    double hh[KCH];
    double ss = 0.0;
#pragma unroll
    for (int i = 0; i < KCH; ++i) {
        hh[i] = i < k ? h[i] : 0.0;
        ss += hh[i] * hh[i];
    }
    const double nrm2 = fmax(h[k] - ss, 0.0);
    const double inv = 1.0 / sqrt(nrm2);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *nrm2_out = nrm2;
        if (nrm2_host) *nrm2_host = nrm2;
    }
    double mx[1] = {0.0};
    const int64_t np = n >> 1;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < np; e += (int64_t)gridDim.x * blockDim.x) {
        double2 we = ld2_nt(w, e);
        double2 v[KCH];
#pragma unroll
        for (int i = 0; i < KCH; ++i)
            if (i < k) v[i] = ld2_stream(V + (int64_t)i * ld, e);
#pragma unroll
        for (int i = 0; i < KCH; ++i)
            if (i < k) {
                we.x -= hh[i] * v[i].x;
                we.y -= hh[i] * v[i].y;
            }
        we.x *= inv;
        we.y *= inv;
        st2_nt(y, e, we);
        mx[0] = fmax(mx[0], fmax(2 * e < n_max ? fabs(we.x) : 0.0, 2 * e + 1 < n_max ? fabs(we.y) : 0.0));
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        const int64_t e = n - 1;
        double we = w[e];
#pragma unroll
        for (int i = 0; i < KCH; ++i)
            if (i < k) we -= hh[i] * V[(int64_t)i * ld + e];
        we *= inv;
        y[e] = we;
        if (e < n_max) mx[0] = fmax(mx[0], fabs(we));
    }
    block_reduce_store(mx, 1, part, 1);
}

void run_update_scale(const double* V, int64_t ld, int k, const double* h, const double* w, double* y, int64_t n,
                      double* nrm2_out, double* part, double* scale_out, hipStream_t s, double* nrm2_host,
                      int64_t n_max) {
    if (n_max < 0 || n_max > n) n_max = n;
    if (k < 1 || k > KCH) throw Error(IIM_E_INVALID_ARG, "update_scale: 1..12 vectors");
    check_vec(V, ld);
    check_vec(w, 0);
    check_vec(y, 0);
    hipLaunchKernelGGL(k_update_scale, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, V, ld, k, h, w, y, n, n_max,
                       nrm2_out, nrm2_host, part);
    IIM_LAUNCH_CHECK();
    final_sum(part, 1, scale_out, s, 1);
}

static int stream_blocks(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(n / 2 + 1, 256), 8192)); }

__global__ void __launch_bounds__(256) k_normalize(const double* x, const double* nrm2, double* y, int64_t n) {
    const double inv = 1.0 / sqrt(*nrm2);
    const int64_t np = n >> 1;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < np; e += (int64_t)gridDim.x * blockDim.x) {
        double2 v = ld2(x, e);
        v.x *= inv;
        v.y *= inv;
        st2(y, e, v);
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) y[n - 1] = x[n - 1] * inv;
}

void run_normalize(const double* x, const double* nrm2, double* y, int64_t n, hipStream_t s) {
    check_vec(x, 0);
    check_vec(y, 0);
    hipLaunchKernelGGL(k_normalize, dim3(stream_blocks(n)), dim3(256), 0, s, x, nrm2, y, n);
    IIM_LAUNCH_CHECK();
}

__global__ void __launch_bounds__(256) k_axpy_multi(const double* Z, int64_t ld, int k, const double* y, double* x,
                                                    int64_t n) {
    double yy[KCH];
#pragma unroll
    for (int i = 0; i < KCH; ++i) yy[i] = i < k ? y[i] : 0.0;
    const int64_t np = n >> 1;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < np; e += (int64_t)gridDim.x * blockDim.x) {
        double2 v = ld2(x, e);
#pragma unroll
        for (int i = 0; i < KCH; ++i)
            if (i < k) {
                const double2 z = ld2_stream(Z + (int64_t)i * ld, e);
                v.x += yy[i] * z.x;
                v.y += yy[i] * z.y;
            }
        st2(x, e, v);
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
        double v = x[n - 1];
#pragma unroll
        for (int i = 0; i < KCH; ++i)
            if (i < k) v += yy[i] * Z[(int64_t)i * ld + n - 1];
        x[n - 1] = v;
    }
}

void run_axpy_multi(const double* Z, int64_t ld, int k, const double* y, double* x, int64_t n, hipStream_t s) {
    if (k == 0) return;
    if (k > KCH) throw Error(IIM_E_INVALID_ARG, "axpy_multi: too many vectors");
    check_vec(Z, ld);
    check_vec(x, 0);
    hipLaunchKernelGGL(k_axpy_multi, dim3(stream_blocks(n)), dim3(256), 0, s, Z, ld, k, y, x, n);
    IIM_LAUNCH_CHECK();
}

__global__ void __launch_bounds__(256) k_axpby(double a, const double* x, double b, double* y, int64_t n) {
    const int64_t np = n >> 1;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < np; e += (int64_t)gridDim.x * blockDim.x) {
        const double2 u = ld2(x, e);
        double2 v = ld2(y, e);
        v.x = a * u.x + b * v.x;
        v.y = a * u.y + b * v.y;
        st2(y, e, v);
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) y[n - 1] = a * x[n - 1] + b * y[n - 1];
}

void run_axpby(double a, const double* x, double b, double* y, int64_t n, hipStream_t s) {
    check_vec(x, 0);
    check_vec(y, 0);
    hipLaunchKernelGGL(k_axpby, dim3(stream_blocks(n)), dim3(256), 0, s, a, x, b, y, n);
    IIM_LAUNCH_CHECK();
}

void run_copy(const double* x, double* y, int64_t n, hipStream_t s) {
    IIM_HIP(hipMemcpyAsync(y, x, n * sizeof(double), hipMemcpyDeviceToDevice, s));
}

__global__ void __launch_bounds__(RED_THREADS) k_absmax(const double* x, int64_t n, double* part) {
    double v[1] = {0.0};
    const int64_t np = n >> 1;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < np; e += (int64_t)gridDim.x * blockDim.x) {
        const double2 u = ld2(x, e);
        v[0] = fmax(v[0], fmax(fabs(u.x), fabs(u.y)));
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) v[0] = fmax(v[0], fabs(x[n - 1]));
    block_reduce_store(v, 1, part, 1);
}

void run_absmax(const double* x, int64_t n, double* part, double* out, hipStream_t s) {
    check_vec(x, 0);
    hipLaunchKernelGGL(k_absmax, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, x, n, part);
    IIM_LAUNCH_CHECK();
    final_sum(part, 1, out, s, 1);
}

__global__ void __launch_bounds__(RED_THREADS) k_norm2(const double* x, int64_t n, double* part) {
    double acc[1] = {0.0};
    const int64_t np = n >> 1;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < np; e += (int64_t)gridDim.x * blockDim.x) {
        const double2 u = ld2(x, e);
        acc[0] += u.x * u.x;
        acc[0] += u.y * u.y;
    }
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) acc[0] += x[n - 1] * x[n - 1];
    block_reduce_store(acc, 1, part, 0);
}

void run_norm2(const double* x, int64_t n, double* part, double* out, hipStream_t s) {
    check_vec(x, 0);
    hipLaunchKernelGGL(k_norm2, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, x, n, part);
    IIM_LAUNCH_CHECK();
    final_sum(part, 1, out, s);
}

// Bordered operator of a singular pure-Neumann problem (Sec. 2.3: the system
// [L 1; 1^T 0] [u; alpha] = [b; gamma]).  After y = L x over the box, this adds
// the shift alpha to every unknown of y and writes y[n] = sum of x over the
// unknowns (deterministic: fixed grid, fixed reduction order).  alpha is read
// from *alpha_src and stored into x[n]: the preconditioner is the identity on
// alpha, so z_j inherits it from v_j here instead of in a launch of its own
// (alpha_src = x + n when x already holds it).  labels: level-0 box labels;
// n: box size, so x and y hold n + 1 entries.
__global__ void __launch_bounds__(RED_THREADS) k_border(double* x, const double* alpha_src, const uint8_t* labels,
                                                        int64_t n, double* y, double* part) {
    double acc[1] = {0.0};
    const double alpha = *alpha_src;
    const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t0 == 0 && alpha_src != x + n) x[n] = alpha;
    for (int64_t e = t0; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        if (is_unknown(labels[e])) {
            acc[0] += x[e];
            y[e] += alpha;
        }
    }
    block_reduce_store(acc, 1, part, 0);
}

void run_border(double* x, const double* alpha_src, const uint8_t* labels, int64_t n, double* y, double* part,
                hipStream_t s) {
    hipLaunchKernelGGL(k_border, dim3(RED_BLOCKS), dim3(RED_THREADS), 0, s, x, alpha_src, labels, n, y, part);
    IIM_LAUNCH_CHECK();
    final_sum(part, 1, y + n, s);
}

}  // namespace iim
