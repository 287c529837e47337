// rpy_lma.hip -- the low-memory form of the diffusion-tensor product
// (arXiv:1203.6208, section "Low memory algorithm"): nothing of size N x N is
// stored; every product recomputes the real-space sum (self term, M1 over
// the images within r_c, the overlap form below 2a) from a cell list, and
// takes the reciprocal sum from the structure factors of its input as the
// stored form does.  Requires max(r_c, 2a) < L/3, so that cells of that side
// number at least 3 per axis and the 27 cells around a bead's cell hold every
// bead any of whose images is within reach (each pair then has one such image
// at most).
#include "rpy_internal.h"
#include "rpy_sf.h"

namespace rpy {

// out[j][k] = in[j][beads[k]] (3 components), j < m: positions or vectors in
// cell order.
__global__ void k_lma_gather(int N, int m, int n3, const int *__restrict__ beads,
                             const double *__restrict__ in, double *__restrict__ out,
                             const int *__restrict__ gate)
{
    if (gate && *gate) return;   // a product past the settled adaptive order
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m * N) return;
    const int j = e / N, k = e % N;
    const int b = beads[k];
    const double *src = in + (size_t)j * n3 + 3 * (size_t)b;
    double *dst = out + (size_t)j * n3 + 3 * (size_t)k;
    dst[0] = src[0];
    dst[1] = src[1];
    dst[2] = src[2];
}

void launch_lma_build(const Ctx &c, hipStream_t s)
{
    launch_cell_list_into(c.N, c.L, c.lma_nc, c.rt, c.lma_start, c.lma_beads, s);
    hipLaunchKernelGGL(k_lma_gather, dim3((c.N + 255) / 256), dim3(256), 0, s, c.N, 1, c.n3,
                       c.lma_beads, c.rt, c.rt_sorted, nullptr);
}

// Real-space product, matrix-free.  Workgroup: 16 consecutive beads in cell
// order, one wave per 4 of them.  For a home bead h (sorted index) the 64
// lanes walk the 27 cells around its cell, each cell's beads in order, and
// test each candidate k cheaply (minimum-image |d|^2 against r_c^2 and
// (2a)^2, the test add_image applies to that image, or k = h); the
// candidates that pass are appended to a per-wave LDS queue (ballot +
// prefix count), and whenever 64 are queued every lane evaluates one of
// them: the 3 x 3 pair block of its minimum image (the self term for k = h)
// times v_k.  Only about a sixth of the stencil is within
// reach, so the expensive pair terms run on full waves.  The lanes are
// combined by a fixed xor tree; the result goes to part slot 0 at the bead's
// own index.  Every step of the walk is deterministic.
constexpr int LMA_HOMES = 16;
constexpr int LMA_QCAP = 128;

__device__ inline void lma_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// The block of one queued pair.  With max(r_c, 2a) < L/3 only the minimum
// image of a pair can be within reach (any other is farther than 2L/3), and
// a bead has no image of itself within reach: the block is add_image of the
// minimum image (the term pair_block would sum), or the self term.
template <int M>
__device__ inline void lma_pair(double hx, double hy, double hz, int k, int h,
                                const PairConst &p, const double *__restrict__ rt_s,
                                const double *__restrict__ vs, int n3, int j0,
                                double acc[M][3])
{
    double b[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (k == h) {
        b[0] = b[3] = b[5] = p.self_coeff;
    } else {
        double dx = hx - rt_s[3 * (size_t)k], dy = hy - rt_s[3 * (size_t)k + 1],
               dz = hz - rt_s[3 * (size_t)k + 2];
        dx -= p.L * rint(dx * p.invL);
        dy -= p.L * rint(dy * p.invL);
        dz -= p.L * rint(dz * p.invL);
        add_image(dx, dy, dz, p, b);
    }
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const double *v = vs + (size_t)(j0 + j) * n3 + 3 * (size_t)k;
        const double v0 = v[0], v1 = v[1], v2 = v[2];
        acc[j][0] += b[0] * v0 + b[1] * v1 + b[2] * v2;
        acc[j][1] += b[1] * v0 + b[3] * v1 + b[4] * v2;
        acc[j][2] += b[2] * v0 + b[4] * v1 + b[5] * v2;
    }
}

// Four waves per SIMD (at most 128 VGPRs; the compiler spills a few values
// to scratch) ran the N = 32000 product 1.3x faster than the three that 169
// VGPRs allow; five or six waves were slower.
template <int M>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_lma_real(int N, int n3, int n3pad, int rhs_cap, int j0,
                                                  double L, int nc, PairConst p,
                                                  const int *__restrict__ start,
                                                  const int *__restrict__ beads,
                                                  const double *__restrict__ rt_s,
                                                  const double *__restrict__ vs,
                                                  double *__restrict__ part,
                                                  const int *__restrict__ gate)
{
    __shared__ int queue[4][LMA_QCAP];
    if (gate && *gate) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int *q = queue[w];
    const double invL = 1.0 / L;
    for (int i = 0; i < LMA_HOMES / 4; ++i) {
        const int h = blockIdx.x * LMA_HOMES + 4 * w + i;   // wave-uniform
        if (h >= N) break;
        const double hx = rt_s[3 * (size_t)h], hy = rt_s[3 * (size_t)h + 1],
                     hz = rt_s[3 * (size_t)h + 2];
        int cx = (int)(hx / L * nc), cy = (int)(hy / L * nc), cz = (int)(hz / L * nc);
        cx = min(max(cx, 0), nc - 1);
        cy = min(max(cy, 0), nc - 1);
        cz = min(max(cz, 0), nc - 1);
        double acc[M][3];
#pragma unroll
        for (int j = 0; j < M; ++j) acc[j][0] = acc[j][1] = acc[j][2] = 0.0;
        int qn = 0;   // queued candidates (wave-uniform)
        for (int cq = 0; cq < 27; ++cq) {
            const int ex = (cx + cq % 3 - 1 + nc) % nc, ey = (cy + (cq / 3) % 3 - 1 + nc) % nc,
                      ez = (cz + cq / 9 - 1 + nc) % nc;
            const int cc = (ez * nc + ey) * nc + ex;
            const int k0 = start[cc], k1 = start[cc + 1];
            for (int base = k0; base < k1; base += 64) {
                const int k = base + lane;
                bool in = false;
                if (k < k1) {
                    double dx = hx - rt_s[3 * (size_t)k], dy = hy - rt_s[3 * (size_t)k + 1],
                           dz = hz - rt_s[3 * (size_t)k + 2];
                    dx -= L * rint(dx * invL);
                    dy -= L * rint(dy * invL);
                    dz -= L * rint(dz * invL);
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    in = k == h || r2 <= p.rc2 || r2 < p.a2x4;
                }
                const unsigned long long mask = __ballot(in);
                const int before = __popcll(mask & ((1ull << lane) - 1ull));
                if (in) q[qn + before] = k;
                qn += __popcll(mask);
                if (qn >= 64) {   // a full wave of pair terms
                    lma_wave_sync();
                    const int kk = q[lane];
                    const int rest = qn - 64;
                    const int moved = lane < rest ? q[64 + lane] : 0;
                    lma_wave_sync();
                    if (lane < rest) q[lane] = moved;
                    qn = rest;
                    lma_pair<M>(hx, hy, hz, kk, h, p, rt_s, vs, n3, j0, acc);
                }
            }
        }
        lma_wave_sync();
        if (lane < qn) lma_pair<M>(hx, hy, hz, q[lane], h, p, rt_s, vs, n3, j0, acc);
        lma_wave_sync();   // the queue is reused by the next home bead
        const int nu = beads[h];
#pragma unroll
        for (int j = 0; j < M; ++j)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double v = acc[j][c];
#pragma unroll
                for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
                if (lane == 0) part[(size_t)(j0 + j) * n3pad + 3 * (size_t)nu + c] = v;
            }
    }
}

void launch_lma_real(const Ctx &c, const double *v, int m, hipStream_t s)
{
    hipLaunchKernelGGL(k_lma_gather, dim3((m * c.N + 255) / 256), dim3(256), 0, s, c.N, m, c.n3,
                       c.lma_beads, v, c.v_sorted, c.gate);
    const dim3 g((c.N + LMA_HOMES - 1) / LMA_HOMES);
#define RPY_LMA_REAL(MC)                                                                        \
    hipLaunchKernelGGL(k_lma_real<MC>, g, dim3(256), 0, s, c.N, c.n3, c.n3pad, c.rhs_cap, j0, \
                       c.L, c.lma_nc, c.pc, c.lma_start, c.lma_beads, c.rt_sorted, c.v_sorted, \
                       c.part, c.gate)
    for (int j0 = 0; j0 < m;) {   // groups of 4, 2, 1 vectors
        const int mc = (m - j0) >= 4 ? 4 : (m - j0) >= 2 ? 2 : 1;
        if (mc == 4) RPY_LMA_REAL(4);
        else if (mc == 2) RPY_LMA_REAL(2);
        else RPY_LMA_REAL(1);
        j0 += mc;
    }
#undef RPY_LMA_REAL
}

// Structure-factor partials of the m input vectors (one or two at a time).
__global__ __launch_bounds__(256) void k_lma_sf(int N, int n3, int nk, int nmax, int rhs_cap,
                                                int nkb, int m, const KVec *__restrict__ kvec,
                                                const double2 *__restrict__ etab,
                                                const double *__restrict__ v,
                                                double *__restrict__ sfpart,
                                                const int *__restrict__ gate)
{
    extern __shared__ double smem[];
    if (gate && *gate) return;
    for (int j0 = 0; j0 < m; j0 += 2) {
        if (j0 > 0) __syncthreads();   // the vector slots are rewritten
        if (m - j0 >= 2)
            sf_partial_block<2>(blockIdx.x, nkb, N, n3, nk, nmax, rhs_cap, j0, kvec, etab, v,
                                sfpart, smem, j0 == 0);
        else
            sf_partial_block<1>(blockIdx.x, nkb, N, n3, nk, nmax, rhs_cap, j0, kvec, etab, v,
                                sfpart, smem, j0 == 0);
    }
}

void launch_lma_sf(const Ctx &c, const double *v, int m, hipStream_t s)
{
    const int nkb = (c.nk + 255) / 256;
    const size_t lds = sizeof(double) * (size_t)(2 * SF_BEADS * 3 * (c.nmax + 1) + SF_BEADS * 2 * 3);
    hipLaunchKernelGGL(k_lma_sf, dim3(c.nsfc * nkb), dim3(256), lds, s, c.N, c.n3, c.nk, c.nmax,
                       c.rhs_cap, nkb, m, c.kvec, c.etab, v, c.sfpart, c.gate);
}

}  // namespace rpy
