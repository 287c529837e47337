// rpy_lanczos.hip -- eigenvalue bounds of D by the Lanczos recurrence, and
// the re-summation used by the adaptive Chebyshev order (arXiv:1203.6208,
// section "Decomposition of the diffusion tensor": the interval must satisfy
// d_max >= lambda_max and d_min <= lambda_min; N_Ch from eq. nint, increased
// until E_f < tol).
#include "rpy_internal.h"

namespace rpy {

constexpr int LZ_THREADS = 1024;

// Fixed-order sum of a per-thread value over one 1024-thread workgroup.
__device__ inline double block_sum(double v, double *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int h = LZ_THREADS / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    const double s = red[0];
    __syncthreads();
    return s;
}

// Per-thread partial sums over i = tid, tid + 1024, ... in ascending order.
// q = r / |r| (one workgroup).
__global__ __launch_bounds__(LZ_THREADS) void k_lanczos_init(int n, const double *__restrict__ r,
                                                             double *__restrict__ q)
{
    __shared__ double red[LZ_THREADS];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += LZ_THREADS) s += r[i] * r[i];
    const double inv = 1.0 / sqrt(block_sum(s, red));
    for (int i = threadIdx.x; i < n; i += LZ_THREADS) q[i] = r[i] * inv;
}

// One Lanczos step after w = D q (one workgroup):
//   w -= beta_{j-1} q_prev;  alpha_j = q . w;  w -= alpha_j q;
//   beta_j = |w|;  q_prev <- w / beta_j  (the next q; buffers rotate)
// ab[2j] = alpha_j, ab[2j + 1] = beta_j; beta_{j-1} = ab[2j - 1] (0 for j = 0).
// A zero beta_j (invariant subspace) leaves q_prev = 0.
__global__ __launch_bounds__(LZ_THREADS) void k_lanczos_step(int n, int j,
                                                             const double *__restrict__ q,
                                                             double *__restrict__ w,
                                                             double *__restrict__ qprev,
                                                             double *__restrict__ ab)
{
    __shared__ double red[LZ_THREADS];
    const double bprev = j > 0 ? ab[2 * j - 1] : 0.0;
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += LZ_THREADS) {
        const double wi = w[i] - (j > 0 ? bprev * qprev[i] : 0.0);
        w[i] = wi;
        s += q[i] * wi;
    }
    const double alpha = block_sum(s, red);
    s = 0.0;
    for (int i = threadIdx.x; i < n; i += LZ_THREADS) {
        const double wi = w[i] - alpha * q[i];
        w[i] = wi;
        s += wi * wi;
    }
    const double beta = sqrt(block_sum(s, red));
    const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
    for (int i = threadIdx.x; i < n; i += LZ_THREADS) qprev[i] = w[i] * inv;
    if (threadIdx.x == 0) {
        ab[2 * j] = alpha;
        ab[2 * j + 1] = beta;
    }
}

void launch_lanczos_init(int n, const double *r, double *q, hipStream_t s)
{
    hipLaunchKernelGGL(k_lanczos_init, dim3(1), dim3(LZ_THREADS), 0, s, n, r, q);
}

void launch_lanczos_step(int n, int j, const double *q, double *w, double *qprev, double *ab,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_lanczos_step, dim3(1), dim3(LZ_THREADS), 0, s, n, j, q, w, qprev, ab);
}

// out = (c_0 / 2) V_0 + sum_{p = 1}^{n_cheb - 1} c_p V_p (p ascending), with
// V_p = vh + p * pstride, m vectors of n3 each; c_p = scal[8 + p].
__global__ void k_cheb_resum(int n3, int m, int n_cheb, size_t pstride,
                             const double *__restrict__ scal, const double *__restrict__ vh,
                             double *__restrict__ out)
{
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)m * n3) return;
    double y = 0.5 * scal[8] * vh[e];
    for (int p = 1; p < n_cheb; ++p) y += scal[8 + p] * vh[(size_t)p * pstride + e];
    out[e] = y;
}

void launch_cheb_resum(int n3, int m, int n_cheb, size_t pstride, const double *scal,
                       const double *vh, double *out, hipStream_t s)
{
    const size_t n = (size_t)m * n3;
    hipLaunchKernelGGL(k_cheb_resum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n3, m,
                       n_cheb, pstride, scal, vh, out);
}

}  // namespace rpy
