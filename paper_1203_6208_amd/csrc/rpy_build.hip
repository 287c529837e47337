// rpy_build.hip -- wrapping, Fourier phase tables and the real-space tiles
// of the diffusion matrix (eq. DF / DFmodified of arXiv:1203.6208).
#include "rpy_internal.h"

namespace rpy {

// One thread per bead: wrapped position rt = L (r/L - floor(r/L)) and the
// phase table e^{i 2 pi j s_a}, j = 0..nmax, for each axis a (s = r/L wrapped).
// A non-finite coordinate raises flags[0] and is replaced by 0 so that every
// later kernel still runs on finite data.
__global__ void k_wrap_tables(int N, double L, int nmax, const double *__restrict__ pos,
                              double *__restrict__ rt, double *__restrict__ sfr,
                              double2 *__restrict__ etab, int *__restrict__ flags)
{
    const int nu = blockIdx.x * blockDim.x + threadIdx.x;
    if (nu >= N) return;
    bool bad = false;
    for (int i = 0; i < 3; ++i) {
        double r = pos[3 * nu + i];
        if (!isfinite(r)) {
            bad = true;
            r = 0.0;
        }
        double s = r / L;
        s = s - floor(s);
        rt[3 * nu + i] = L * s;
        sfr[3 * nu + i] = s;
        double2 *tab = etab + (size_t)(3 * nu + i) * (nmax + 1);
        for (int j = 0; j <= nmax; ++j) {
            double sn, cs;
            sincospi(2.0 * j * s, &sn, &cs);
            tab[j] = make_double2(cs, sn);
        }
    }
    if (bad) atomicOr(flags, 1);
}

void launch_wrap_tables(const Ctx &c, const double *pos, hipStream_t s)
{
    const int bs = 256;
    hipLaunchKernelGGL(k_wrap_tables, dim3((c.N + bs - 1) / bs), dim3(bs), 0, s, c.N, c.L,
                       c.nmax, pos, c.rt, c.sfr, c.etab, c.flags);
}

// Wrapped positions only; a non-finite coordinate raises flags[0] as above.
__global__ void k_wrap_positions(int N, double L, const double *__restrict__ pos,
                                 double *__restrict__ rt, int *__restrict__ flags)
{
    const int nu = blockIdx.x * blockDim.x + threadIdx.x;
    if (nu >= N) return;
    bool bad = false;
    for (int i = 0; i < 3; ++i) {
        double r = pos[3 * nu + i];
        if (!isfinite(r)) {
            bad = true;
            r = 0.0;
        }
        const double s = r / L;
        rt[3 * nu + i] = L * (s - floor(s));
    }
    if (bad) atomicOr(flags, 1);
}

void launch_wrap_positions(const Ctx &c, const double *pos, double *rt, hipStream_t s)
{
    const int bs = 256;
    hipLaunchKernelGGL(k_wrap_positions, dim3((c.N + bs - 1) / bs), dim3(bs), 0, s, c.N, c.L, pos,
                       rt, c.flags);
}

__device__ inline uint16_t to_bf16(double d)
{
    // round-to-nearest-even of the float value
    const float f = (float)d;
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// One workgroup per stored tile (I <= J).  Thread (bi0, bj) computes the
// pair blocks (I*64 + bi0 + 4s, J*64 + bj), s = 0..15, over all periodic
// images and writes the 3x3 block into the row-major tile; LOWP also writes
// the FP32 (1) or BF16 (2) copy of the same tile.
template <int LOWP>
__global__ __launch_bounds__(256) void k_build_tiles(int N, const int2 *__restrict__ tile_ij,
                                                     const double *__restrict__ rt, PairConst p,
                                                     double *__restrict__ d64,
                                                     float *__restrict__ d32,
                                                     uint16_t *__restrict__ d16)
{
    __shared__ double sI[TS], sJ[TS];
    const int t = blockIdx.x;
    const int2 ij = tile_ij[t];
    const int I = ij.x, J = ij.y;
    const int tid = threadIdx.x;
    for (int e = tid; e < TS; e += blockDim.x) {
        const int bI = I * TB + e / 3, bJ = J * TB + e / 3;
        sI[e] = bI < N ? rt[3 * (size_t)I * TB + e] : 0.0;
        sJ[e] = bJ < N ? rt[3 * (size_t)J * TB + e] : 0.0;
    }
    __syncthreads();
    const int bj = tid & (TB - 1);
    const int bi0 = tid >> 6;
    const int mu = J * TB + bj;
    for (int s = 0; s < TB / 4; ++s) {
        const int bi = bi0 + 4 * s;
        const int nu = I * TB + bi;
        double b[6] = {0, 0, 0, 0, 0, 0};
        if (nu < N && mu < N) {
            pair_block(sI[3 * bi] - sJ[3 * bj], sI[3 * bi + 1] - sJ[3 * bj + 1],
                       sI[3 * bi + 2] - sJ[3 * bj + 2], nu == mu, p, b);
        }
        // packed FP64 planes: a wave writes 512 contiguous bytes per plane
        const size_t o6 = (size_t)t * TILE6 + (size_t)bi * 6 * TB + bj;
#pragma unroll
        for (int e = 0; e < 6; ++e) d64[o6 + (size_t)e * TB] = b[e];
        if (LOWP) {
            const double v[9] = {b[0], b[1], b[2], b[1], b[3], b[4], b[2], b[4], b[5]};
            const size_t o = (size_t)t * TILE_ELEMS + (size_t)(3 * bi) * TS + 3 * bj;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    if (LOWP == 1) d32[o + (size_t)i * TS + j] = (float)v[3 * i + j];
                    if (LOWP == 2) d16[o + (size_t)i * TS + j] = to_bf16(v[3 * i + j]);
                }
            }
        }
    }
}

void launch_build_tiles(const Ctx &c, hipStream_t s)
{
    if (c.lma) {   // low-memory form: only the cell list and sorted positions
        launch_lma_build(c, s);
        return;
    }
    const dim3 g(c.ntiles), b(256);
    if (c.lowp == RPY_PREC_F32)
        hipLaunchKernelGGL(k_build_tiles<1>, g, b, 0, s, c.N, c.tile_ij, c.rt, c.pc, c.d64,
                           c.d32, c.d16);
    else if (c.lowp == RPY_PREC_BF16)
        hipLaunchKernelGGL(k_build_tiles<2>, g, b, 0, s, c.N, c.tile_ij, c.rt, c.pc, c.d64,
                           c.d32, c.d16);
    else
        hipLaunchKernelGGL(k_build_tiles<0>, g, b, 0, s, c.N, c.tile_ij, c.rt, c.pc, c.d64,
                           c.d32, c.d16);
}

// Dense row-major copy of the stored FP64 real-space matrix (test helper).
__global__ void k_dense_copy(int n3, int nbt, const double *__restrict__ d64,
                             double *__restrict__ out)
{
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)n3 * n3) return;
    int row = (int)(idx / n3), col = (int)(idx % n3);
    int I = row / TS, J = col / TS, r = row % TS, cc = col % TS;
    if (I > J) {   // the transposed block: the same, each block being symmetric
        int t = I; I = J; J = t;
        t = r; r = cc; cc = t;
    }
    const size_t tidx = (size_t)I * nbt - (size_t)I * (I - 1) / 2 + (J - I);
    const int a = min(r % 3, cc % 3), b = max(r % 3, cc % 3);
    const int plane = 3 * a - a * (a - 1) / 2 + (b - a);   // xx xy xz yy yz zz
    out[idx] = d64[tidx * TILE6 + ((size_t)(r / 3) * 6 + plane) * TB + cc / 3];
}

void launch_dense_copy(const Ctx &c, double *out, hipStream_t s)
{
    const size_t n = (size_t)c.n3 * c.n3;
    hipLaunchKernelGGL(k_dense_copy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, c.n3,
                       c.nbt, c.d64, out);
}

}  // namespace rpy
