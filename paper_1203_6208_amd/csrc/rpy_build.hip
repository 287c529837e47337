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

// One workgroup per stored tile (I <= J).  Wave w takes the bead rows
// bi = w + 4 s (s = 0..15), its 64 lanes the bead columns bj, so each step
// computes 64 pair blocks (I*64 + bi, J*64 + bj) over their periodic images.
// Whenever every axis has at most two candidate image shifts (always when
// max(r_c, 2a) < L), a pair's candidates are the corners ci = 4 ix + 2 iy +
// iz of a 2 x 2 x 2 cube (valid if ix < nxc, iy < nyc, iz < nzc; the order
// nx, ny, nz of pair_block).  The lanes test their candidates
// cheaply (|d|^2 against r_c^2 and (2a)^2), append those that contribute to
// a per-wave LDS queue (ballot + prefix count) and evaluate the queue 64 at a
// time, so the erfc / exp work runs on full waves (without the queue every
// lane waits for the costliest candidate of all 64 lanes, about eight
// evaluations per pair).  Each lane then adds its images' terms in candidate
// order (the operations of pair_block, so the block is bit-identical).  A
// step in which some pair has three or more shifts on an axis falls back to
// pair_block.  The block goes to the packed FP64 planes; LOWP also writes
// packed FP32 (1) or BF16 (2) planes.
constexpr int IMG_SLOTS = 8;
constexpr int IMG_QCAP = 128;

__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int LOWP>
__global__ __launch_bounds__(256) void k_build_tiles(int N, const int2 *__restrict__ tile_ij,
                                                     const double *__restrict__ rt, PairConst p,
                                                     double *__restrict__ d64,
                                                     float *__restrict__ p32,
                                                     uint16_t *__restrict__ p16)
{
    __shared__ double sI[TS], sJ[TS];
    __shared__ double q_r2[4][IMG_QCAP];
    __shared__ int q_id[4][IMG_QCAP];
    __shared__ double2 res[4][IMG_SLOTS][64];   // (c1, c2) of lane's candidate
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
    const int lane = tid & 63, w = tid >> 6;
    const int bj = lane;
    const int mu = J * TB + bj;
    double *qr = q_r2[w];
    int *qi = q_id[w];
    for (int s = 0; s < TB / 4; ++s) {
        const int bi = w + 4 * s;
        const int nu = I * TB + bi;
        const bool live = nu < N && mu < N;
        const bool self = nu == mu;
        const double d0x = sI[3 * bi] - sJ[3 * bj], d0y = sI[3 * bi + 1] - sJ[3 * bj + 1],
                     d0z = sI[3 * bi + 2] - sJ[3 * bj + 2];
        const int xl = image_lo(d0x, p), yl = image_lo(d0y, p), zl = image_lo(d0z, p);
        const int nxc = max(0, image_hi(d0x, p) - xl + 1), nyc = max(0, image_hi(d0y, p) - yl + 1),
                  nzc = max(0, image_hi(d0z, p) - zl + 1);
        double b[6] = {0, 0, 0, 0, 0, 0};
        if (__any(live && (nxc > 2 || nyc > 2 || nzc > 2))) {   // wave-uniform: the plain walk
            if (live) pair_block(d0x, d0y, d0z, self, p, b);
        } else {
            const double dxs[2] = {d0x + xl * p.L, d0x + (xl + 1) * p.L};
            const double dys[2] = {d0y + yl * p.L, d0y + (yl + 1) * p.L};
            const double dzs[2] = {d0z + zl * p.L, d0z + (zl + 1) * p.L};
            unsigned inmask = 0u;   // this lane's contributing candidates
            int qn = 0;             // wave-uniform
#pragma unroll
            for (int ci = 0; ci < IMG_SLOTS; ++ci) {
                const int ix = ci >> 2, iy = (ci >> 1) & 1, iz = ci & 1;
                const double dx = dxs[ix], dy = dys[iy], dz = dzs[iz];
                const double r2 = dx * dx + dy * dy + dz * dz;
                const bool in = live && ix < nxc && iy < nyc && iz < nzc &&
                                !(self && xl + ix == 0 && yl + iy == 0 && zl + iz == 0) &&
                                (r2 <= p.rc2 || r2 < p.a2x4);
                inmask |= in ? 1u << ci : 0u;
                const unsigned long long mask = __ballot(in);
                const int before = __popcll(mask & ((1ull << lane) - 1ull));
                if (in) {
                    qr[qn + before] = r2;
                    qi[qn + before] = ci * 64 + lane;
                }
                qn += __popcll(mask);
                if (qn >= 64) {   // a full wave of image terms
                    wave_sync();
                    const double er2 = qr[lane];
                    const int eid = qi[lane];
                    const int rest = qn - 64;
                    const double mr2 = lane < rest ? qr[64 + lane] : 0.0;
                    const int mid = lane < rest ? qi[64 + lane] : 0;
                    wave_sync();
                    if (lane < rest) {
                        qr[lane] = mr2;
                        qi[lane] = mid;
                    }
                    qn = rest;
                    double c1, c2;
                    image_coeffs(er2, p, c1, c2);
                    res[w][eid >> 6][eid & 63] = make_double2(c1, c2);
                }
            }
            wave_sync();
            if (lane < qn) {
                double c1, c2;
                image_coeffs(qr[lane], p, c1, c2);
                const int eid = qi[lane];
                res[w][eid >> 6][eid & 63] = make_double2(c1, c2);
            }
            wave_sync();
#pragma unroll
            for (int ci = 0; ci < IMG_SLOTS; ++ci) {   // this lane's images, in order
                if (!(inmask & (1u << ci))) continue;
                const double dx = dxs[ci >> 2], dy = dys[(ci >> 1) & 1], dz = dzs[ci & 1];
                const double r2 = dx * dx + dy * dy + dz * dz;
                const double2 cc = res[w][ci][lane];
                add_coeffs(dx, dy, dz, r2, cc.x, cc.y, b);
            }
            if (self) {
                b[0] += p.self_coeff;
                b[3] += p.self_coeff;
                b[5] += p.self_coeff;
            }
            wave_sync();   // res and the queue are reused by the next step
        }
        // packed planes: a wave writes 512 contiguous bytes per FP64 plane
        const size_t o6 = (size_t)t * TILE6 + (size_t)bi * 6 * TB + bj;
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            d64[o6 + (size_t)e * TB] = b[e];
            if (LOWP == 1) p32[o6 + (size_t)e * TB] = (float)b[e];
            if (LOWP == 2) p16[o6 + (size_t)e * TB] = to_bf16(b[e]);
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
                           c.p32, c.p16);
    else if (c.lowp == RPY_PREC_BF16)
        hipLaunchKernelGGL(k_build_tiles<2>, g, b, 0, s, c.N, c.tile_ij, c.rt, c.pc, c.d64,
                           c.p32, c.p16);
    else
        hipLaunchKernelGGL(k_build_tiles<0>, g, b, 0, s, c.N, c.tile_ij, c.rt, c.pc, c.d64,
                           c.p32, c.p16);
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
