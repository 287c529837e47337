// rpy_grad.hip -- reverse mode of u = D(R) F + p(D(R)) dW, the drift product
// plus the Chebyshev sum of arXiv:1203.6208 (eq. DF, eq. cheb1-cheb3) on a
// fixed interval.
//
// With g = dL/du the adjoint vectors of the recurrence are
//   mu_p = c_p g + 2 Y mu_{p+1} - mu_{p+2}   (p = N_Ch - 1 .. 1, mu_{N_Ch} = mu_{N_Ch+1} = 0)
// and dL = sum_q x_q^T dD y_q over the pairs (x_q, y_q) = (g, F),
// (ya mu_1, V_0), (2 ya mu_p, V_{p-1}) for p >= 2, ya = 2/(d_max - d_min).
// D's pair block depends on d = r_l - r_m only and is even in d, so
//   dL/dr_l = sum_{m != l} grad_d [ W_lm : D(d) ],  W = sum_q x_q y_q^T + y_q x_q^T,
// split into the real-space images (pair_grad, per stored tile of W) and the
// reciprocal sum
//   -sum_k k sum_q [ x_q,l . (sin T^C_k(y_q) - cos T^S_k(y_q))
//                  + y_q,l . (sin T^C_k(x_q) - cos T^S_k(x_q)) ]
// with T^C_k(v) = 2 m(k) (I - khat khat) sum_m cos(k.r_m) v_m (and T^S with
// sin), i.e. the T_k of a forward product of v.  Self terms and the images of
// a bead with itself do not move with r_l.
#include "rpy_internal.h"
#include "rpy_sf.h"

namespace rpy {

// mu_p = c_p g and x_p = xs ya mu_p (the first adjoint vector needs no product).
__global__ void k_adj_init(int n3, int p, double xs, const double *__restrict__ scal,
                           const double *__restrict__ g, double *__restrict__ mu,
                           double *__restrict__ xq)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n3) return;
    const double m = scal[8 + p] * g[i];
    mu[i] = m;
    xq[i] = xs * scal[2] * m;
}

void launch_adj_init(const Ctx &c, int p, double xs, const double *g, double *mu, double *xq,
                     hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_init, dim3((c.n3 + 255) / 256), dim3(256), 0, s, c.n3, p, xs,
                       c.scal, g, mu, xq);
}

__global__ void k_add(double *out, const double *a, const double *b, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[i] + b[i];
}

void launch_add(double *out, const double *a, const double *b, size_t n, hipStream_t s)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, a, b, n);
}

// ------------------------------------------------------------------ W tiles
// W = sum_q x_q y_q^T + y_q x_q^T on the stored tiles (I <= J), row-major
// TS x TS per tile.  This is a product of rank K = 2 nq,
//   W_IJ = A_I B_J,  A_I[r][2q + s] = (x_q, y_q)_s[rows of I],
//                    B_J[2q + s][c] = (y_q, x_q)_s[rows of J],
// run on FP64 16x16x4 matrix-core instructions.  One workgroup per tile and
// group of WCOL columns; the K index is staged in LDS WKC at a time (the
// slices of A and of the group's part of B, zero past 3N and past K; every
// load of a slice is issued before the first LDS write); wave w owns the
// 16 x 16 blocks of block rows 3 w .. 3 w + 2 and the group's block columns.
// Narrow groups and short slices keep the registers few (160 VGPRs at
// WCOL = 64, WKC = 8), so that two waves share each SIMD: at N = 2000 this
// runs in 68 us against 156 us for the same product on the vector units and
// 114 us with 96-column groups and WKC = 16.
// Operand layout of v_mfma_f64_16x16x4f64 (lane = 16 g + i): A[row i][k g],
// B[k g][col i]; the result holds rows g + 4 e of column i, e = 0..3.
constexpr int WKC = 8;
constexpr int WCOL = 64;
constexpr int WSPLIT = TS / WCOL;
constexpr int WNBC = WCOL / 16;
typedef double d4v_w __attribute__((ext_vector_type(4)));
static_assert(WKC * TS % 256 == 0 && WKC * WCOL % 256 == 0,
              "the W-tile slices are staged 256 values at a time");
__global__ __launch_bounds__(256) void k_grad_wtiles(int n3, int nq, const int2 *__restrict__ tile_ij,
                                                     const double *__restrict__ xy,
                                                     double *__restrict__ wt)
{
    __shared__ double sa[WKC][TS], sb[WKC][WCOL];
    const int t = blockIdx.x / WSPLIT, part = blockIdx.x % WSPLIT;
    const int2 ij = tile_ij[t];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane >> 4, i = lane & 15;
    const int K = 2 * nq;
    const size_t rowI = (size_t)ij.x * TS, rowJ = (size_t)ij.y * TS + WCOL * part;
    double *tile = wt + (size_t)t * TILE_ELEMS + WCOL * part;
    d4v_w acc[3][WNBC];
#pragma unroll
    for (int R = 0; R < 3; ++R)
#pragma unroll
        for (int C = 0; C < WNBC; ++C) acc[R][C] = d4v_w{0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += WKC) {
        constexpr int PA = WKC * TS / 256, PB = WKC * WCOL / 256;
        double va[PA], vb[PB];
#pragma unroll
        for (int u = 0; u < PA; ++u) {
            const int e = (int)threadIdx.x + 256 * u;
            const int kk = e / TS, r = e % TS, k = min(k0 + kk, K - 1);
            va[u] = xy[(size_t)k * n3 + min(rowI + r, (size_t)n3 - 1)];
        }
#pragma unroll
        for (int u = 0; u < PB; ++u) {
            const int e = (int)threadIdx.x + 256 * u;
            const int kk = e / WCOL, r = e % WCOL, k = min(k0 + kk, K - 1);
            vb[u] = xy[(size_t)(k ^ 1) * n3 + min(rowJ + r, (size_t)n3 - 1)];
        }
        __syncthreads();   // the previous slice has been used
#pragma unroll
        for (int u = 0; u < PA; ++u) {
            const int e = (int)threadIdx.x + 256 * u;
            const int kk = e / TS, r = e % TS;
            sa[kk][r] = k0 + kk < K && rowI + r < (size_t)n3 ? va[u] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < PB; ++u) {
            const int e = (int)threadIdx.x + 256 * u;
            const int kk = e / WCOL, r = e % WCOL;
            sb[kk][r] = k0 + kk < K && rowJ + r < (size_t)n3 ? vb[u] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < WKC; kk += 4) {
            double av[3];
#pragma unroll
            for (int R = 0; R < 3; ++R) av[R] = sa[kk + g][16 * (3 * w + R) + i];
#pragma unroll
            for (int C = 0; C < WNBC; ++C) {
                const double bv = sb[kk + g][16 * C + i];
#pragma unroll
                for (int R = 0; R < 3; ++R)
                    acc[R][C] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[R], bv, acc[R][C], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int R = 0; R < 3; ++R)
#pragma unroll
        for (int C = 0; C < WNBC; ++C)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                tile[(size_t)(16 * (3 * w + R) + g + 4 * e) * TS + 16 * C + i] = acc[R][C][e];
}

void launch_grad_wtiles(const Ctx &c, int nq, hipStream_t s)
{
    hipLaunchKernelGGL(k_grad_wtiles, dim3(WSPLIT * c.ntiles), dim3(256), 0, s, c.n3, nq, c.tile_ij,
                       c.xy, c.wgrad);
}

// ------------------------------------------------------- real-space gradient
// One workgroup per stored tile (I, J): lane = bead m of J, wave w takes the
// beads l = w, w + 4, ... of I.  Each (l, m) with l != m reads its 3 x 3
// block of W (coalesced across the lanes), symmetrises it and sums the image
// gradients.  Row sums (over the lanes, fixed xor tree) give the
// contribution to bead l -> gpart[J][3 l + c]; on off-diagonal tiles the
// negated pair terms summed over l (per lane, then the 4 waves in order) give
// bead m's -> gpart[I][3 m + c].  Every (slot, row) is written exactly once.
// Two waves per SIMD (at most 256 VGPRs, a few spills) instead of the one
// its 279 VGPRs allow: 128 us against 154 us at N = 2000.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_grad_real(int N, int n3pad, const int2 *__restrict__ tile_ij,
                                                   const double *__restrict__ rt, PairConst p,
                                                   const double *__restrict__ wt,
                                                   double *__restrict__ gpart)
{
    __shared__ double sI[TS], sJ[TS];
    __shared__ double scol[4][TS];
    const int t = blockIdx.x;
    const int2 ij = tile_ij[t];
    const int I = ij.x, J = ij.y;
    for (int e = threadIdx.x; e < TS; e += blockDim.x) {
        const int bI = I * TB + e / 3, bJ = J * TB + e / 3;
        sI[e] = bI < N ? rt[3 * (size_t)I * TB + e] : 0.0;
        sJ[e] = bJ < N ? rt[3 * (size_t)J * TB + e] : 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int mu = J * TB + lane;
    const bool muok = mu < N;
    const double *W = wt + (size_t)t * TILE_ELEMS;
    const bool offd = I != J;
    double cacc[3] = {0.0, 0.0, 0.0};
    for (int s = 0; s < TB / 4; ++s) {
        const int lp = w + 4 * s;
        const int lam = I * TB + lp;
        double gr[3] = {0.0, 0.0, 0.0};
        if (lam < N && muok && (offd || lp != lane)) {
            const double *wr = W + (size_t)(3 * lp) * TS + 3 * lane;
            double w9[9];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) w9[3 * i + j] = wr[(size_t)i * TS + j];
            const double Ws[6] = {w9[0], 0.5 * (w9[1] + w9[3]), 0.5 * (w9[2] + w9[6]),
                                  w9[4], 0.5 * (w9[5] + w9[7]), w9[8]};
            pair_grad(sI[3 * lp] - sJ[3 * lane], sI[3 * lp + 1] - sJ[3 * lane + 1],
                      sI[3 * lp + 2] - sJ[3 * lane + 2], p, Ws, gr);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double v = gr[c];
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
            if (lane == 0 && lam < N) gpart[(size_t)J * n3pad + 3 * lam + c] = v;
            cacc[c] -= gr[c];
        }
    }
    if (!offd) return;
#pragma unroll
    for (int c = 0; c < 3; ++c) scol[w][3 * lane + c] = cacc[c];
    __syncthreads();
    for (int e = threadIdx.x; e < TS; e += blockDim.x)
        gpart[(size_t)I * n3pad + (size_t)J * TS + e] =
            ((scol[0][e] + scol[1][e]) + scol[2][e]) + scol[3][e];
}

void launch_grad_real(const Ctx &c, hipStream_t s)
{
    hipLaunchKernelGGL(k_grad_real, dim3(c.ntiles), dim3(256), 0, s, c.N, c.n3pad, c.tile_ij,
                       c.rt, c.pc, c.wgrad, c.gpart);
}

// ------------------------------------------------ reciprocal-space gradient
// Structure-factor partials of nv (even) vectors v[0 .. nv-1] (stride 3N):
// workgroup (chunk x wave-vector block, y) takes the vectors 4 y .. 4 y + 3
// (a last pair when nv is not a multiple of 4); sfpart as in a forward
// product, for the reduction of launch_sf_reduce.  One group of vectors per
// workgroup keeps 4x more workgroups busy than looping over the groups
// (at N = 2000 the loop ran 96 workgroups on 256 compute units).
__global__ __launch_bounds__(256) void k_grad_sf(int N, int n3, int nk, int nmax, int rhs_cap,
                                                 int nkb, int nv, const KVec *__restrict__ kvec,
                                                 const double2 *__restrict__ etab,
                                                 const double *__restrict__ v,
                                                 double *__restrict__ sfpart)
{
    extern __shared__ double smem[];
    const int j0 = 4 * blockIdx.y;
    if (nv - j0 >= 4)
        sf_partial_block<4>(blockIdx.x, nkb, N, n3, nk, nmax, rhs_cap, j0, kvec, etab, v, sfpart,
                            smem);
    else
        sf_partial_block<2>(blockIdx.x, nkb, N, n3, nk, nmax, rhs_cap, j0, kvec, etab, v, sfpart,
                            smem);
}

void launch_grad_sf(const Ctx &c, const double *v, int nv, hipStream_t s)
{
    const int nkb = (c.nk + 255) / 256;
    const size_t lds = sizeof(double) * (size_t)(2 * SF_BEADS * 3 * (c.nmax + 1) + SF_BEADS * 4 * 3);
    hipLaunchKernelGGL(k_grad_sf, dim3(c.nsfc * nkb, (nv + 3) / 4), dim3(256), lds, s, c.N, c.n3,
                       c.nk, c.nmax, c.rhs_cap, nkb, nv, c.kvec, c.etab, v, c.sfpart);
}

// Per bead l: the reciprocal term above for the nq pairs whose T_k are in
// tk[k][2 qq + (0: x, 1: y)][6].  Workgroup: 4 beads x 64 wave-vector slices
// (lane = bead (low 2 bits) and 16 slices, 4 waves; phases by the n_z
// recursion as in the product's back-projection); slices are combined in a
// fixed order (xor tree over the lanes of a bead, then the 4 waves); gk =
// (or +=, accumulate) the result.
constexpr int GK_BEADS = 4;
constexpr int GK_SLICES = 64;
constexpr int GK_QMAX = 8;
__global__ __launch_bounds__(256) void k_grad_kspace(int N, int n3, int nk, int rhs_cap, int nq,
                                                      double twopi_L, int accumulate,
                                                      const KVec *__restrict__ kvec,
                                                      const double *__restrict__ sfr,
                                                      const double *__restrict__ xy,
                                                      const double *__restrict__ tk,
                                                      double *__restrict__ gk)
{
    __shared__ double red[4][3][GK_BEADS];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int bl = lane & 3, sub = lane >> 2;
    const int u = 16 * w + sub;   // slice 0 .. 63
    const int nu = blockIdx.x * GK_BEADS + bl;
    const bool live = nu < N;
    double xv[GK_QMAX][3], yv[GK_QMAX][3];
#pragma unroll
    for (int q = 0; q < GK_QMAX; ++q)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const bool ok = live && q < nq;
            xv[q][c] = ok ? xy[(size_t)(2 * q) * n3 + 3 * nu + c] : 0.0;
            yv[q][c] = ok ? xy[(size_t)(2 * q + 1) * n3 + 3 * nu + c] : 0.0;
        }
    double acc[3] = {0.0, 0.0, 0.0};
    if (live) {
        const double sx = sfr[3 * nu], sy = sfr[3 * nu + 1], sz = sfr[3 * nu + 2];
        const int klo = (int)((long)u * nk / GK_SLICES),
                  khi = (int)((long)(u + 1) * nk / GK_SLICES);
        double ezr, ezi;
        sincospi(2.0 * sz, &ezi, &ezr);
        double cs = 1.0, sn = 0.0;
        int px = -(1 << 30), py = 0, pz = 0;
        for (int k = klo; k < khi; ++k) {
            const KVec kv = kvec[k];
            if (kv.nx == px && kv.ny == py && kv.nz == pz + 1) {
                const double c2 = cs * ezr - sn * ezi;
                sn = cs * ezi + sn * ezr;
                cs = c2;
            } else {
                sincospi(2.0 * (kv.nx * sx + kv.ny * sy + kv.nz * sz), &sn, &cs);
            }
            px = kv.nx;
            py = kv.ny;
            pz = kv.nz;
            const double *tt = tk + (size_t)k * rhs_cap * 6;
            double sk = 0.0;
#pragma unroll
            for (int q = 0; q < GK_QMAX; ++q) {
                if (q < nq) {
                    const double *tx = tt + 12 * q, *ty = tx + 6;
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        sk += xv[q][c] * (sn * ty[c] - cs * ty[3 + c]) +
                              yv[q][c] * (sn * tx[c] - cs * tx[3 + c]);
                }
            }
            acc[0] -= sk * (twopi_L * kv.nx);
            acc[1] -= sk * (twopi_L * kv.ny);
            acc[2] -= sk * (twopi_L * kv.nz);
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double v = acc[c];
#pragma unroll
        for (int o = 4; o <= 32; o <<= 1) v += __shfl_xor(v, o);
        if (sub == 0) red[w][c][bl] = v;
    }
    __syncthreads();
    if (threadIdx.x < 3 * GK_BEADS) {
        const int b = threadIdx.x / 3, c = threadIdx.x % 3;
        const int bead = blockIdx.x * GK_BEADS + b;
        if (bead < N) {
            double s = 0.0;
#pragma unroll
            for (int ww = 0; ww < 4; ++ww) s += red[ww][c][b];
            const size_t o = 3 * (size_t)bead + c;
            gk[o] = accumulate ? gk[o] + s : s;
        }
    }
}

void launch_grad_kspace(const Ctx &c, const double *xy, int nq, int accumulate, hipStream_t s)
{
    hipLaunchKernelGGL(k_grad_kspace, dim3((c.N + GK_BEADS - 1) / GK_BEADS), dim3(256), 0, s, c.N,
                       c.n3, c.nk, c.rhs_cap, nq, 2.0 * M_PI / c.L, accumulate, c.kvec, c.sfr, xy,
                       c.tk, c.gk);
}

// gpos[3 l + c] = sum over the tile-column slots K (ascending) + reciprocal part.
__global__ void k_grad_sum(int n3, int n3pad, int nbt, const double *__restrict__ gpart,
                           const double *__restrict__ gk, double *__restrict__ gpos)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n3) return;
    double s = 0.0;
    for (int K = 0; K < nbt; ++K) s += gpart[(size_t)K * n3pad + i];
    gpos[i] = s + gk[i];
}

void launch_grad_sum(const Ctx &c, double *gpos, hipStream_t s)
{
    hipLaunchKernelGGL(k_grad_sum, dim3((c.n3 + 255) / 256), dim3(256), 0, s, c.n3, c.n3pad, c.nbt,
                       c.gpart, c.gk, gpos);
}

}  // namespace rpy
