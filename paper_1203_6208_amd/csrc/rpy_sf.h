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

}  // namespace rpy
