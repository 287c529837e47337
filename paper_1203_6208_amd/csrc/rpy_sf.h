// rpy_sf.h -- structure-factor partials of a product's input vectors, shared
// by the tile-product kernels (arXiv:1203.6208, eq. DF, reciprocal sum taken
// per product as S_k = sum_mu {cos, sin}(k.r_mu) v_mu).
#pragma once
#include "rpy_internal.h"

namespace rpy {

// e^{i 2 pi n.s} for bead table tab[3][nmax+1] (n_x >= 0 on the half space).
__device__ inline double2 kphase(const KVec &kv, const double2 *tab, int nm1)
{
    double2 ex = tab[kv.nx];
    double2 ey = tab[nm1 + (kv.ny < 0 ? -kv.ny : kv.ny)];
    double2 ez = tab[2 * nm1 + (kv.nz < 0 ? -kv.nz : kv.nz)];
    if (kv.ny < 0) ey.y = -ey.y;
    if (kv.nz < 0) ez.y = -ez.y;
    const double2 xy = make_double2(ex.x * ey.x - ex.y * ey.y, ex.x * ey.y + ex.y * ey.x);
    return make_double2(xy.x * ez.x - xy.y * ez.y, xy.x * ez.y + xy.y * ez.x);
}

// Structure-factor partials of the product's input vector, carried by the
// first `nsf` workgroups of the product kernel (they only read v, so they
// run beside the tile stream).  Workgroup b: bead chunk b / nkb (SF_BEADS
// beads), wave-vector block b % nkb; one thread per wave vector:
//   sfpart[chunk][6 j + c][k] = sum_mu {cos, sin}(k.r_mu) v_mu,c.
template <int M>
__device__ inline void sf_partial_block(int b, int nkb, int N, int n3, int nk, int nmax,
                                        int rhs_cap, int j0, const KVec *__restrict__ kvec,
                                        const double2 *__restrict__ etab,
                                        const double *__restrict__ v, double *__restrict__ sfpart,
                                        double *smem, bool load_tab = true)
{
    const int nm1 = nmax + 1;
    const int chunk = b / nkb, kb = b % nkb;
    const int b0 = chunk * SF_BEADS;
    const int nb = min(SF_BEADS, N - b0);
    double2 *stab = reinterpret_cast<double2 *>(smem);          // [SF_BEADS][3*nm1]
    double *sv = smem + 2 * SF_BEADS * 3 * nm1;                  // [SF_BEADS][M][3]
    if (load_tab)  // else still in LDS from the previous group of vectors
        for (int e = threadIdx.x; e < nb * 3 * nm1; e += blockDim.x)
            stab[e] = etab[(size_t)b0 * 3 * nm1 + e];
    for (int e = threadIdx.x; e < nb * 3 * M; e += blockDim.x) {
        const int bl = e / (3 * M), r = e % (3 * M), j = r / 3, c = r % 3;
        sv[e] = v[(size_t)(j0 + j) * n3 + 3 * (b0 + bl) + c];
    }
    __syncthreads();
    const int k = kb * blockDim.x + threadIdx.x;
    if (k >= nk) return;  // no barrier follows inside this function
    const KVec kv = kvec[k];
    double acc[M][6];
#pragma unroll
    for (int j = 0; j < M; ++j)
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[j][c] = 0.0;
#pragma unroll 4
    for (int bl = 0; bl < nb; ++bl) {
        const double2 e = kphase(kv, stab + bl * 3 * nm1, nm1);
#pragma unroll
        for (int j = 0; j < M; ++j)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double x = sv[bl * 3 * M + 3 * j + c];
                acc[j][c] += e.x * x;
                acc[j][3 + c] += e.y * x;
            }
    }
    double *o = sfpart + ((size_t)chunk * 6 * rhs_cap + 6 * j0) * nk + k;
#pragma unroll
    for (int j = 0; j < M; ++j)
#pragma unroll
        for (int c = 0; c < 6; ++c) o[(size_t)(6 * j + c) * nk] = acc[j][c];
}

// Structure factors of the product's input vectors by wave vector, carried
// by the first workgroups of the tile-product kernel (they read only the
// positions and v, so they run beside the tile stream).  Workgroup b owns the
// KPW wave vectors KPW b .. KPW b + KPW - 1 and sums over every bead,
//   C_k = sum_mu cos(k.r_mu) v_mu,   S_k = sum_mu sin(k.r_mu) v_mu,
// with k.r_mu = 2 pi n.s_mu (s = r/L of the wrapped position) from sincospi;
// thread t takes the beads t, t + 64 NW, ... and the sums are combined in a
// fixed order (an xor tree inside each wave, then the NW waves in LDS).  The
// workgroup then applies 2 m(k) (I - khat khat) (eq. DF, third term) and
// writes tk[k][j0 + j] = (T^C_k, T^S_k): the sum over beads is complete, so
// no reduction over bead chunks follows.
template <int M> constexpr int sf_kpw() { return M <= 2 ? 2 : 1; }

template <int M, int NW = 4>
__device__ inline void sf_direct_block(int b, int N, int nk, int rhs_cap, int j0, double invL,
                                       int n3, const KVec *__restrict__ kvec,
                                       const KCoef *__restrict__ kcoef,
                                       const double *__restrict__ rt,
                                       const double *__restrict__ v, double *__restrict__ tk,
                                       double *smem)
{
    constexpr int KPW = sf_kpw<M>();
    constexpr int NV = KPW * M * 6;   // sums per thread
    double nxs[KPW], nys[KPW], nzs[KPW];
#pragma unroll
    for (int q = 0; q < KPW; ++q) {
        const KVec kv = kvec[min(KPW * b + q, nk - 1)];
        nxs[q] = 2.0 * kv.nx;
        nys[q] = 2.0 * kv.ny;
        nzs[q] = 2.0 * kv.nz;
    }
    double acc[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = 0.0;
    for (int mu = threadIdx.x; mu < N; mu += blockDim.x) {
        const double sx = rt[3 * mu] * invL, sy = rt[3 * mu + 1] * invL,
                     sz = rt[3 * mu + 2] * invL;
        double x[M][3];
#pragma unroll
        for (int j = 0; j < M; ++j)
#pragma unroll
            for (int c = 0; c < 3; ++c) x[j][c] = v[(size_t)(j0 + j) * n3 + 3 * mu + c];
#pragma unroll
        for (int q = 0; q < KPW; ++q) {
            double sn, cs;
            sincospi(nxs[q] * sx + nys[q] * sy + nzs[q] * sz, &sn, &cs);
#pragma unroll
            for (int j = 0; j < M; ++j)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    acc[(q * M + j) * 6 + c] += cs * x[j][c];
                    acc[(q * M + j) * 6 + 3 + c] += sn * x[j][c];
                }
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double a = acc[i];
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) a += __shfl_xor(a, o);
        if (lane == 0) smem[w * NV + i] = a;
    }
    __syncthreads();
    // thread (q, j, half) of the first 2 KPW M: the NW waves in order, then
    // the projection
    if (threadIdx.x < 2 * KPW * M) {
        const int half = threadIdx.x & 1, qj = threadIdx.x >> 1, q = qj / M, j = qj % M;
        const int k = KPW * b + q;
        if (k < nk) {
            double t[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int i = qj * 6 + 3 * half + c;
                double a = smem[i];
#pragma unroll
                for (int w2 = 1; w2 < NW; ++w2) a += smem[w2 * NV + i];
                t[c] = a;
            }
            const KCoef kc = kcoef[k];
            const double h = kc.hx * t[0] + kc.hy * t[1] + kc.hz * t[2];
            double *o = tk + ((size_t)k * rhs_cap + j0 + j) * 6 + 3 * half;
            o[0] = kc.w * (t[0] - kc.hx * h);
            o[1] = kc.w * (t[1] - kc.hy * h);
            o[2] = kc.w * (t[2] - kc.hz * h);
        }
    }
}

}  // namespace rpy
