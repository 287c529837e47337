// rpy_block.hip -- the block product Y = D.V for up to 16 vectors at once, as
// used by the Chebyshev recurrence (arXiv:1203.6208, eq. cheb1-cheb3: every
// term is one product of D with the current vectors) when the stored
// real-space tiles are FP32 or BF16.
//
//   1. k_pack_block: the vectors in the operand layouts below (low precision
//      for the tiles, FP64 for the reciprocal sum).
//   2. k_block_tiles: real-space tiles on the matrix cores, FP32 accumulation
//      inside a tile, FP32 partial per tile and tile column, stored in blocks
//      of 16 rows: part32[K][row / 16][j][row % 16].
//   3. k_block_sf + k_block_sf_reduce: structure factors S_k = sum_mu e^{i k.r_mu}
//      v_mu as an FP64 matrix-core product of the phase matrix (computed once
//      per set of positions by k_block_phases) with V, then the fixed-order
//      chunk sum and 2 m(k) (I - khat khat) (eq. DF, third term, evaluated
//      per product).
//   4. k_block_epi: the back-projection sum_k (cos, sin)(k.r_nu) T_k as an
//      FP64 matrix-core product, plus the tile partials (summed in a fixed
//      order by extra workgroups of the k_block_sf launch), plus the
//      recurrence step.
// The reciprocal sum and the recurrence are FP64 throughout.
//
// Tile product: each wave owns one stored tile A = A_IJ (192 x 192, I <= J):
//   row product    A   X_J  -> slot J, rows of I
//   column product A^T X_I  -> slot I, rows of J   (I < J only)
// as 16 x 16 MFMA output blocks (16 rows or columns x 16 vectors).  The tile
// is read once, 16 rows (a strip) at a time, with 16-byte loads.  A lane's
// loaded values lie along one tile row, the A-operand layout of the row
// product (operand row = lane % 16).  The column product needs the operand
// row to be a tile column, so each 16 x 16 (FP32) or 16 x 32 (BF16) piece is
// transposed through a small per-wave LDS buffer.  The 12 column blocks stay
// in registers for the whole tile; the waves never synchronise.
#include "rpy_internal.h"

namespace rpy {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));
typedef short s4v __attribute__((ext_vector_type(4)));
typedef uint32_t u4v __attribute__((ext_vector_type(4)));
typedef uint32_t u2v __attribute__((ext_vector_type(2)));

constexpr int TLD32 = 20;      // FP32 transpose buffer row stride (floats)
constexpr int TLD16 = 40;      // BF16 transpose buffer row stride (bf16)
constexpr int SF_WAVES = 4;    // waves per structure-factor workgroup

__device__ inline uint16_t bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Packed vectors, zero beyond n3 and beyond m:
//   FP32: xq[r / 4][j][r % 4]
//   BF16: xh[r / 8][j][r % 8] = bf16(x), xl[...] = bf16(x - xh) (a hi + lo
//         pair: the operand carries about 16 significant bits of x)
//   FP64: vpk[r][j]
// so that a lane's operand for 4 (8) consecutive rows of one vector is a
// single 16-byte load, and 16 lanes read 16 vectors of one row together.
__global__ void k_pack_block(int n3, int n3pad, int m, int bf16, const double *__restrict__ v,
                             void *__restrict__ xpk, double *__restrict__ vpk,
                             const int *__restrict__ gate)
{
    if (gate && *gate) return;   // a product past the settled adaptive order
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n3pad * BLOCK_RHS) return;
    {
        const int r = o >> 4, j = o & 15;
        vpk[o] = (j < m && r < n3) ? v[(size_t)j * n3 + r] : 0.0;
    }
    int r, j;
    if (bf16) {
        r = (o >> 7) * 8 + (o & 7);
        j = (o >> 3) & 15;
    } else {
        r = (o >> 6) * 4 + (o & 3);
        j = (o >> 2) & 15;
    }
    const double x = (j < m && r < n3) ? v[(size_t)j * n3 + r] : 0.0;
    if (bf16) {
        uint16_t *xh = reinterpret_cast<uint16_t *>(xpk);
        const uint16_t h = bf16_rne((float)x);
        const double hv = (double)__uint_as_float((uint32_t)h << 16);
        xh[o] = h;
        xh[(size_t)n3pad * BLOCK_RHS + o] = bf16_rne((float)(x - hv));
    } else {
        reinterpret_cast<float *>(xpk)[o] = (float)x;
    }
}

// Orders this wave's LDS writes before its following LDS reads (and the
// reads before the next overwrite).  Only lanes of one wave share a buffer.
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------- FP32
// Half strip (R, h): rows 16R .. 16R + 15, columns 96h .. 96h + 95, six
// chunks C = 6h + c of 16 columns.  Lane (g = lane / 16, i = lane % 16) holds
// A[16R + i][16C + 4g + s], s = 0..3.  Row product step s: operand row i,
// k = g <-> column 16C + 4g + s, B = X_J[16C + 4g + s][i].  Column product
// step s (after the transpose): operand row i <-> column 16C + i,
// k = g <-> row 16R + 4g + s, B = X_I[16R + 4g + s][i].  The loads of a
// half strip are X_I for its rows (first half only) then its 6 tile pieces,
// so that waiting for them never waits for a later prefetch.
constexpr int RING32 = 3;      // half strips in flight per wave (FP32)
constexpr int RING16 = 4;      // strips in flight per wave (BF16)

struct Half32 {
    f4v xi;
    f4v a[6];
};

__device__ inline void load_half32(const float *tile, const float *xq, int rowI, int q, int i,
                                   int g, Half32 &s)
{
    const int R = q >> 1, h = q & 1;
    if (h == 0)
        s.xi = *reinterpret_cast<const f4v *>(xq + (size_t)((rowI + 16 * R) / 4 + g) * 64 + 4 * i);
    const float *row = tile + (size_t)(16 * R + i) * TS + 96 * h + 4 * g;
#pragma unroll
    for (int c = 0; c < 6; ++c) s.a[c] = *reinterpret_cast<const f4v *>(row + 16 * c);
}

// racc[2]: two accumulators (even and odd chunks) halve the dependent chain.
__device__ inline void half32(const Half32 &s, const f4v &xi, int h, bool offd, int i, int g,
                              const f4v *xj, float *tb, f4v *cacc, f4v *racc)
{
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const int C = 6 * h + c;
        const f4v a = s.a[c];
        f4v &ra = racc[c & 1];
        ra = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, xj[C].x, ra, 0, 0, 0);
        ra = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, xj[C].y, ra, 0, 0, 0);
        ra = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, xj[C].z, ra, 0, 0, 0);
        ra = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, xj[C].w, ra, 0, 0, 0);
        if (offd) {
            *reinterpret_cast<f4v *>(tb + i * TLD32 + 4 * g) = a;
            wave_lds_sync();
            const float t0 = tb[(4 * g + 0) * TLD32 + i];
            const float t1 = tb[(4 * g + 1) * TLD32 + i];
            const float t2 = tb[(4 * g + 2) * TLD32 + i];
            const float t3 = tb[(4 * g + 3) * TLD32 + i];
            wave_lds_sync();
            cacc[C] = __builtin_amdgcn_mfma_f32_16x16x4f32(t0, xi.x, cacc[C], 0, 0, 0);
            cacc[C] = __builtin_amdgcn_mfma_f32_16x16x4f32(t1, xi.y, cacc[C], 0, 0, 0);
            cacc[C] = __builtin_amdgcn_mfma_f32_16x16x4f32(t2, xi.z, cacc[C], 0, 0, 0);
            cacc[C] = __builtin_amdgcn_mfma_f32_16x16x4f32(t3, xi.w, cacc[C], 0, 0, 0);
        }
    }
}

// ---------------------------------------------------------------- BF16
// Strip R, chunk C (32 columns): lane holds A[16R + i][32C + 8g + e],
// e = 0..7 (one 16-byte load).  Row product: elements 0..3 and 4..7 are two
// K = 16 operands with k = 4g + e <-> column 32C + 8g + e (+4), B = the
// matching rows of X_J (hi and lo parts, FP32 accumulate).  Column product
// for the column half h: operand row i <-> column 32C + 16h + i,
// k = 4g + e <-> row 16R + 4g + e.
struct Strip16 {
    u2v xih, xil;
    u4v a[TS / 32];
};

__device__ inline void load_strip16(const uint16_t *tile, const uint16_t *xh,
                                    const uint16_t *xl, int rowI, int R, int i, int g,
                                    Strip16 &s)
{
    const size_t xo = (size_t)((rowI + 16 * R) / 8 + (g >> 1)) * 128 + 8 * i + 4 * (g & 1);
    s.xih = *reinterpret_cast<const u2v *>(xh + xo);
    s.xil = *reinterpret_cast<const u2v *>(xl + xo);
    const uint16_t *row = tile + (size_t)(16 * R + i) * TS + 8 * g;
#pragma unroll
    for (int C = 0; C < TS / 32; ++C) s.a[C] = *reinterpret_cast<const u4v *>(row + 32 * C);
}

__device__ inline s4v as_s4(uint32_t x, uint32_t y)
{
    return __builtin_bit_cast(s4v, u2v{x, y});
}

__device__ inline void strip16(const Strip16 &s, int R, bool offd, int i, int g,
                               const u4v *xjh, const u4v *xjl, uint16_t *tb, f4v *cacc,
                               float *prow, bool store)
{
    const s4v xih = as_s4(s.xih.x, s.xih.y), xil = as_s4(s.xil.x, s.xil.y);
    f4v racc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
#pragma unroll
    for (int C = 0; C < TS / 32; ++C) {
        const u4v a = s.a[C];
        const s4v a0 = as_s4(a.x, a.y), a1 = as_s4(a.z, a.w);
        f4v &ra = racc[C & 1];
        ra = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, as_s4(xjh[C].x, xjh[C].y), ra, 0, 0, 0);
        ra = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, as_s4(xjl[C].x, xjl[C].y), ra, 0, 0, 0);
        ra = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, as_s4(xjh[C].z, xjh[C].w), ra, 0, 0, 0);
        ra = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, as_s4(xjl[C].z, xjl[C].w), ra, 0, 0, 0);
        if (offd) {
            *reinterpret_cast<u4v *>(tb + i * TLD16 + 8 * g) = a;
            wave_lds_sync();
            uint32_t t[2][2];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const uint16_t *q = tb + (4 * g) * TLD16 + 16 * h + i;
                t[h][0] = (uint32_t)q[0] | ((uint32_t)q[TLD16] << 16);
                t[h][1] = (uint32_t)q[2 * TLD16] | ((uint32_t)q[3 * TLD16] << 16);
            }
            wave_lds_sync();
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const s4v at = as_s4(t[h][0], t[h][1]);
                f4v &cc = cacc[2 * C + h];
                cc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(at, xih, cc, 0, 0, 0);
                cc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(at, xil, cc, 0, 0, 0);
            }
        }
    }
    if (store) *reinterpret_cast<f4v *>(prow + 256 * R) = racc[0] + racc[1];
}

// Wave w of workgroup b takes stored tile 4 b + w.  The strip loop is fully
// unrolled so that the ring of prefetched strips lives in registers and the
// load waits stay per strip.
template <int BF16>
__global__ __launch_bounds__(256) void k_block_tiles(int n3pad, int m, int ntiles,
                                                     const int2 *__restrict__ tile_ij,
                                                     const void *__restrict__ tiles,
                                                     const void *__restrict__ xpk,
                                                     float *__restrict__ part,
                                                     const int *__restrict__ gate)
{
    __shared__ float tbuf[4 * 16 * (BF16 ? TLD16 / 2 : TLD32)];
    if (gate && *gate) return;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = lane & 15, g = lane >> 4;
    const int t = (int)blockIdx.x * 4 + w;
    if (t >= ntiles) return;
    const int2 ij = tile_ij[t];
    const int I = ij.x, J = ij.y;
    const bool offd = I != J;
    const bool store = i < m;
    // output blocks of 16 rows x 16 vectors are contiguous (1 KB): row block
    // I*12 + R of slot J (row product), J*12 + C of slot I (column product);
    // lane (g, i) holds rows 4g .. 4g + 3 of vector i
    const int nrb = n3pad / 16;
    float *prow = part + ((size_t)J * nrb + I * (TS / 16)) * 256 + 16 * i + 4 * g;
    float *pcol = part + ((size_t)I * nrb + J * (TS / 16)) * 256 + 16 * i + 4 * g;
    f4v cacc[TS / 16];
#pragma unroll
    for (int C = 0; C < TS / 16; ++C) cacc[C] = f4v{0.f, 0.f, 0.f, 0.f};
    if (!BF16) {
        const float *tile = reinterpret_cast<const float *>(tiles) + (size_t)t * TILE_ELEMS;
        const float *xq = reinterpret_cast<const float *>(xpk);
        float *tb = tbuf + w * 16 * TLD32;
        f4v xj[TS / 16];
#pragma unroll
        for (int C = 0; C < TS / 16; ++C)
            xj[C] = *reinterpret_cast<const f4v *>(xq + (size_t)((J * TS + 16 * C) / 4 + g) * 64 + 4 * i);
        constexpr int NQ = 2 * (TS / 16);   // half strips per tile
        Half32 ring[RING32];
#pragma unroll
        for (int q = 0; q < RING32 - 1; ++q) load_half32(tile, xq, I * TS, q, i, g, ring[q]);
        f4v xi = {0.f, 0.f, 0.f, 0.f};
        f4v racc[2];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            if (q + RING32 - 1 < NQ)
                load_half32(tile, xq, I * TS, q + RING32 - 1, i, g, ring[(q + RING32 - 1) % RING32]);
            const int h = q & 1;
            if (h == 0) {
                xi = ring[q % RING32].xi;
                racc[0] = racc[1] = f4v{0.f, 0.f, 0.f, 0.f};
            }
            half32(ring[q % RING32], xi, h, offd, i, g, xj, tb, cacc, racc);
            if (h == 1 && store)
                *reinterpret_cast<f4v *>(prow + 256 * (q >> 1)) = racc[0] + racc[1];
        }
    } else {
        const uint16_t *tile = reinterpret_cast<const uint16_t *>(tiles) + (size_t)t * TILE_ELEMS;
        const uint16_t *xh = reinterpret_cast<const uint16_t *>(xpk);
        const uint16_t *xl = xh + (size_t)n3pad * BLOCK_RHS;
        uint16_t *tb = reinterpret_cast<uint16_t *>(tbuf) + w * 16 * TLD16;
        u4v xjh[TS / 32], xjl[TS / 32];
#pragma unroll
        for (int C = 0; C < TS / 32; ++C) {
            const size_t o = (size_t)((J * TS + 32 * C) / 8 + g) * 128 + 8 * i;
            xjh[C] = *reinterpret_cast<const u4v *>(xh + o);
            xjl[C] = *reinterpret_cast<const u4v *>(xl + o);
        }
        Strip16 ring[RING16];
#pragma unroll
        for (int R = 0; R < RING16 - 1; ++R) load_strip16(tile, xh, xl, I * TS, R, i, g, ring[R]);
#pragma unroll
        for (int R = 0; R < TS / 16; ++R) {
            if (R + RING16 - 1 < TS / 16)
                load_strip16(tile, xh, xl, I * TS, R + RING16 - 1, i, g,
                             ring[(R + RING16 - 1) % RING16]);
            strip16(ring[R % RING16], R, offd, i, g, xjh, xjl, tb, cacc, prow, store);
        }
    }
    if (offd && store) {
#pragma unroll
        for (int C = 0; C < TS / 16; ++C)
            *reinterpret_cast<f4v *>(pcol + 256 * C) = cacc[C];
    }
}

void launch_block_tiles(const Ctx &c, int prec, const double *v, int m, hipStream_t s)
{
    const int bf16 = prec == RPY_PREC_BF16;
    const int np = c.n3pad * BLOCK_RHS;
    hipLaunchKernelGGL(k_pack_block, dim3((np + 255) / 256), dim3(256), 0, s, c.n3, c.n3pad, m,
                       bf16, v, c.xpk, c.vpk, c.gate);
    const dim3 grid((c.ntiles + 3) / 4);
    if (bf16)
        hipLaunchKernelGGL(k_block_tiles<1>, grid, dim3(256), 0, s, c.n3pad, m, c.ntiles,
                           c.tile_ij, (const void *)c.d16, (const void *)c.xpk, c.part32, c.gate);
    else
        hipLaunchKernelGGL(k_block_tiles<0>, grid, dim3(256), 0, s, c.n3pad, m, c.ntiles,
                           c.tile_ij, (const void *)c.d32, (const void *)c.xpk, c.part32, c.gate);
}

// ------------------------------------------------- structure factors (FP64)
// Phase matrix eph[q][k][r] = e^{i k.r_mu}, mu = 4 q + r, k < nk16 (nk rounded
// up to 16; zero for k >= nk and for mu >= N, so no lane needs a select),
// from the per-axis tables etab[mu][3][nmax + 1] (n_x >= 0 on the half space;
// negative n_y, n_z conjugate).  Computed once per set of positions and read
// by both matrix-core passes of every block product.
__global__ void k_block_phases(int N, int nk, int nk16, int nmax, const KVec *__restrict__ kvec,
                               const double2 *__restrict__ etab, double2 *__restrict__ eph)
{
    const size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int nq = (N + 3) / 4;
    if (o >= (size_t)nq * nk16 * 4) return;
    const int r = (int)(o & 3);
    const int k = (int)((o >> 2) % nk16);
    const int mu = (int)((o >> 2) / nk16) * 4 + r;
    double2 e = make_double2(0.0, 0.0);
    if (mu < N && k < nk) {
        const int nm1 = nmax + 1;
        const KVec kv = kvec[k];
        const double2 *tab = etab + (size_t)mu * 3 * nm1;
        double2 ex = tab[kv.nx];
        double2 ey = tab[nm1 + (kv.ny < 0 ? -kv.ny : kv.ny)];
        double2 ez = tab[2 * nm1 + (kv.nz < 0 ? -kv.nz : kv.nz)];
        if (kv.ny < 0) ey.y = -ey.y;
        if (kv.nz < 0) ez.y = -ez.y;
        const double xr = ex.x * ey.x - ex.y * ey.y, xi = ex.x * ey.y + ex.y * ey.x;
        e = make_double2(xr * ez.x - xi * ez.y, xr * ez.y + xi * ez.x);
    }
    eph[o] = e;
}

void launch_block_phases(const Ctx &c, hipStream_t s)
{
    const int nk16 = (c.nk + 15) / 16 * 16;
    const size_t n = (size_t)((c.N + 3) / 4) * nk16 * 4;
    hipLaunchKernelGGL(k_block_phases, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, c.N,
                       c.nk, nk16, c.nmax, c.kvec, c.etab, c.eph);
}

// Workgroup (k block of 16 wave vectors, chunk of bead quads); wave w takes
// the quads w, w + 4, ... of the chunk.  Per quad, lane (g, i) holds the
// phase of k = k0 + i and bead 4 q + g (the A operand of both products: row
// = k, inner index = bead) and V[4 q + g][c][j = i] (the B operand), both
// loaded 3 quads ahead; six 16x16x4 FP64 MFMAs add
//   sum_mu {cos, sin}(k.r_mu) v_{mu c j}.
// The waves are summed in a fixed order through LDS and wave 0 writes the
// block's partial sums contiguously:
//   sfpart[k block][chunk][6 j + 3 half + c][k % 16].
struct SfLd {
    double2 e;
    double x[3];
};
// The streamed operands are not declared __restrict__: loads the compiler may
// treat as invariant get rematerialised at their use, which undoes the
// prefetch.
// Workgroups past the structure-factor grid (blockIdx.x >= nkb) sum the
// tile partials instead, 16 beads each (3 row blocks of 16 rows x 16
// vectors, contiguous per slot K): 16 slots per batch of independent loads,
// summed pairwise inside a batch and batch after batch in K order, into
// ypart[j][row].  This HBM stream overlaps the matrix-core work.
__device__ inline void block_part_sum(int b, int N, int n3, int n3pad, int m, int nslot,
                                      const float *__restrict__ part, double *__restrict__ ypart)
{
    const int nu0 = 16 * b, nb = min(16, N - nu0);
    const int nrb = n3pad / 16;
    for (int o = threadIdx.x; o < BLOCK_RHS * 48; o += blockDim.x) {
        const int rbl = o >> 8, j = (o >> 4) & 15, rr = o & 15;
        const int r = 16 * rbl + rr;     // row of the 48
        if (r >= 3 * nb || j >= m) continue;
        const float *pp = part + (size_t)(3 * b + rbl) * 256 + 16 * j + rr;
        const size_t ks = (size_t)nrb * 256;
        double y = 0.0;
        int K = 0;
        for (; K + 16 <= nslot; K += 16) {
            float q[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) q[u] = pp[(K + u) * ks];
            double t[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) t[u] = (double)q[2 * u] + (double)q[2 * u + 1];
            y += ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
        }
        for (; K < nslot; ++K) y += (double)pp[K * ks];
        ypart[(size_t)j * n3 + 3 * nu0 + r] = y;
    }
}

__global__ __launch_bounds__(256) void k_block_sf(int nk, int nk16, int nq, int cq, int nkb,
                                                  int N, int n3, int n3pad, int m, int nslot,
                                                  const double2 *eph, const double *vpk,
                                                  double *sfpart,
                                                  const float *__restrict__ part,
                                                  double *__restrict__ ypart,
                                                  const int *__restrict__ gate)
{
    __shared__ d4v red[SF_WAVES - 1][6][64];
    if (gate && *gate) return;
    if ((int)blockIdx.x >= nkb) {
        const int b = (blockIdx.x - nkb) + blockIdx.y * (gridDim.x - nkb);
        if (16 * b < N) block_part_sum(b, N, n3, n3pad, m, nslot, part, ypart);
        return;
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = lane & 15, g = lane >> 4;
    const int k0 = blockIdx.x * 16, ch = blockIdx.y;
    const int q0 = ch * cq, q1 = min(nq, q0 + cq);
    const int k = k0 + i;
    d4v acc[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) acc[q] = d4v{0.0, 0.0, 0.0, 0.0};
    // Branch-free: indices are clamped to valid entries (a quad past the
    // chunk is loaded but never consumed); phases of k >= nk are stored as
    // zero.  A conditional load here would make the compiler wait for every
    // outstanding load at the join.
    auto fetch = [&](int q, SfLd &d) {
        const int qs = min(q, nq - 1);
        d.e = eph[((size_t)qs * nk16 + k) * 4 + g];
        const double *xv = vpk + (size_t)(12 * qs + 3 * g) * BLOCK_RHS + i;
        d.x[0] = xv[0];
        d.x[1] = xv[BLOCK_RHS];
        d.x[2] = xv[2 * BLOCK_RHS];
    };
    // Ring of 4 buffers in fixed registers (loop unrolled by 4): buffer b
    // is loaded 3 steps before it is consumed.  A step past the chunk
    // consumes a zero phase.
    auto use = [&](const SfLd &d, int q) {
        const bool on = q < q1;
        const double c = on ? d.e.x : 0.0, sn = on ? d.e.y : 0.0;
        acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(c, d.x[0], acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(c, d.x[1], acc[1], 0, 0, 0);
        acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(c, d.x[2], acc[2], 0, 0, 0);
        acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(sn, d.x[0], acc[3], 0, 0, 0);
        acc[4] = __builtin_amdgcn_mfma_f64_16x16x4f64(sn, d.x[1], acc[4], 0, 0, 0);
        acc[5] = __builtin_amdgcn_mfma_f64_16x16x4f64(sn, d.x[2], acc[5], 0, 0, 0);
    };
    constexpr int S = SF_WAVES;
    SfLd b0, b1, b2, b3;
    const int qa = q0 + w;
    fetch(qa, b0);
    fetch(qa + S, b1);
    fetch(qa + 2 * S, b2);
    for (int q = qa; q < q1; q += 4 * S) {
        // compiler-only barriers keep each prefetch where it is written (the
        // loaded values are otherwise forwarded and the loads re-issued
        // where they are consumed)
        fetch(q + 3 * S, b3);
        __asm__ volatile("" ::: "memory");
        use(b0, q);
        fetch(q + 4 * S, b0);
        __asm__ volatile("" ::: "memory");
        use(b1, q + S);
        fetch(q + 5 * S, b1);
        __asm__ volatile("" ::: "memory");
        use(b2, q + 2 * S);
        fetch(q + 6 * S, b2);
        __asm__ volatile("" ::: "memory");
        use(b3, q + 3 * S);
    }
    if (w > 0)
#pragma unroll
        for (int q = 0; q < 6; ++q) red[w - 1][q][lane] = acc[q];
    __syncthreads();
    if (w > 0) return;
#pragma unroll
    for (int q = 0; q < 6; ++q)
#pragma unroll
        for (int ww = 0; ww < SF_WAVES - 1; ++ww) acc[q] += red[ww][q][lane];
    // FP64 MFMA output: lane holds rows g + 4e (wave vectors) of column i
    // (vector j = i)
    double *o = sfpart + ((size_t)blockIdx.x * gridDim.y + ch) * 6 * BLOCK_RHS * 16;
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int q = 0; q < 6; ++q) o[(6 * i + q) * 16 + g + 4 * e] = acc[q][e];
}

// Chunk sum in chunk order and T_k = 2 m(k) (I - khat khat) (C_k or S_k) for
// one (k, vector, cos/sin half) per thread, written as tkm[k][3 half + c][j].
// Thread (k block, 2 j + half, k % 16); the chunks of one k block lie
// together, 16 x 96 doubles apart.
__global__ void k_block_sf_reduce(int nk, int nch, const KCoef *__restrict__ kcoef,
                                  const double *__restrict__ sfpart, double *__restrict__ tkm,
                                  const int *__restrict__ gate)
{
    if (gate && *gate) return;
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    const int kb = o / (2 * BLOCK_RHS * 16), r = o % (2 * BLOCK_RHS * 16);
    const int q2 = r >> 4, kk = r & 15;           // q2 = 2 j + half
    const int k = 16 * kb + kk;
    if (k >= nk) return;
    const int j = q2 >> 1, half = q2 & 1;
    const size_t cst = (size_t)6 * BLOCK_RHS * 16;
    const double *src = sfpart + (size_t)kb * nch * cst + (6 * j + 3 * half) * 16 + kk;
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
#pragma unroll 4
    for (int ch = 0; ch < nch; ++ch) {
        t0 += src[ch * cst];
        t1 += src[ch * cst + 16];
        t2 += src[ch * cst + 32];
    }
    const KCoef kc = kcoef[k];
    const double h = kc.hx * t0 + kc.hy * t1 + kc.hz * t2;
    double *d = tkm + (size_t)k * 6 * BLOCK_RHS + 3 * half * BLOCK_RHS + j;
    d[0] = kc.w * (t0 - kc.hx * h);
    d[BLOCK_RHS] = kc.w * (t1 - kc.hy * h);
    d[2 * BLOCK_RHS] = kc.w * (t2 - kc.hz * h);
}

void launch_block_sf(const Ctx &c, int m, hipStream_t s)
{
    const int nq = (c.N + 3) / 4;
    const int cq = (nq + c.nchb - 1) / c.nchb;
    const int nkb = (c.nk + 15) / 16;
    // grid x: nkb structure-factor blocks, then ceil(npg / nchb) part-sum
    // workgroups per grid row (npg = 16-bead groups)
    const int npg = (c.N + 15) / 16;
    const int px = (npg + c.nchb - 1) / c.nchb;
    hipLaunchKernelGGL(k_block_sf, dim3(nkb + px, c.nchb), dim3(64 * SF_WAVES), 0, s, c.nk,
                       (c.nk + 15) / 16 * 16, nq, cq, nkb, c.N, c.n3, c.n3pad, m, c.nbt, c.eph,
                       c.vpk, c.sfpart, c.part32, c.ypart, c.gate);
    const int nt = (c.nk + 15) / 16 * 2 * BLOCK_RHS * 16;
    hipLaunchKernelGGL(k_block_sf_reduce, dim3((nt + 255) / 256), dim3(256), 0, s, c.nk, c.nchb,
                       c.kcoef, c.sfpart, c.tkm, c.gate);
}

// ------------------------------ back-projection + partial sum + epilogue
// Workgroup: 16 beads nu0 .. nu0 + 15, EPI_W waves; wave w takes the
// wave-vector steps w, w + EPI_W, ... (4 wave vectors each).  Lane (g, i)
// holds the phase of bead nu0 + i and k = 4 step + g (A operand: row =
// bead, inner = k) and T[k][3 half + c][j = i] (B operand; tkm rows >= nk are
// zero), loaded 3 steps ahead; six FP64 MFMAs per step add
//   sum_k cos(k.r) Tc + sin(k.r) Ts,  c = 0..2.
// The waves are summed in a fixed order in LDS; thread (j, bead) adds the
// summed tile partials ypart and applies the epilogue of f.mode (as in
// k_kspace_epi).
constexpr int EPI_W = 8;
struct EpiLd {
    double2 e;
    double t[6];
};
__global__ __launch_bounds__(64 * EPI_W) void k_block_epi(int N, int n3, int nk4, int nk16,
                                                          const double2 *eph, const double *tkm,
                                                          const double *__restrict__ ypart,
                                                          EpiArgs f, const int *__restrict__ gate)
{
    __shared__ double red[EPI_W][3][16][17];
    if (gate && *gate) return;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int i = lane & 15, g = lane >> 4;
    const int nu0 = blockIdx.x * 16;
    // dead lanes read a zero entry of the last quad (phases of mu >= N are 0)
    const int nus = min(nu0 + i, ((N + 3) / 4) * 4 - 1);
    const double2 *ep = eph + (size_t)(nus >> 2) * nk16 * 4 + (nus & 3);
    d4v acc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] = d4v{0.0, 0.0, 0.0, 0.0};
    const int nst = nk4 / 4;
    // Branch-free (see k_block_sf): a step past the end is loaded from a
    // valid row and consumes a zero phase; phases of k >= nk are zero.
    auto fetch = [&](int st, EpiLd &d) {
        const int k = 4 * min(st, nst - 1) + g;
        d.e = ep[(size_t)k * 4];
        const double *tr = tkm + (size_t)k * 6 * BLOCK_RHS + i;
#pragma unroll
        for (int q = 0; q < 6; ++q) d.t[q] = tr[q * BLOCK_RHS];
    };
    auto use = [&](const EpiLd &d, int st) {
        const bool on = st < nst;
        const double c = on ? d.e.x : 0.0, sn = on ? d.e.y : 0.0;
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            acc[cc] = __builtin_amdgcn_mfma_f64_16x16x4f64(c, d.t[cc], acc[cc], 0, 0, 0);
            acc[cc] = __builtin_amdgcn_mfma_f64_16x16x4f64(sn, d.t[3 + cc], acc[cc], 0, 0, 0);
        }
    };
    // ring of 4 buffers in fixed registers, as in k_block_sf
    constexpr int S = EPI_W;
    EpiLd b0, b1, b2, b3;
    fetch(w, b0);
    fetch(w + S, b1);
    fetch(w + 2 * S, b2);
    for (int st = w; st < nst; st += 4 * S) {
        fetch(st + 3 * S, b3);
        __asm__ volatile("" ::: "memory");
        use(b0, st);
        fetch(st + 4 * S, b0);
        __asm__ volatile("" ::: "memory");
        use(b1, st + S);
        fetch(st + 5 * S, b1);
        __asm__ volatile("" ::: "memory");
        use(b2, st + 2 * S);
        fetch(st + 6 * S, b2);
        __asm__ volatile("" ::: "memory");
        use(b3, st + 3 * S);
    }
    // FP64 MFMA output: lane holds beads g + 4e of vector i
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) red[w][c][g + 4 * e][i] = acc[c][e];
    __syncthreads();
    if (threadIdx.x >= 256) return;
    const int j = threadIdx.x >> 4, bl = threadIdx.x & 15;
    const int bead = nu0 + bl;
    if (bead >= N || j >= f.m) return;
    const double ya = f.scal ? f.scal[2] : 0.0, yb = f.scal ? f.scal[3] : 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double yk = 0.0;
#pragma unroll
        for (int ww = 0; ww < EPI_W; ++ww) yk += red[ww][c][bl][j];
        const size_t o = (size_t)j * n3 + 3 * bead + c;
        const double yy = yk + ypart[o];
        if (f.mode == EPI_APPLY) {
            f.vout[o] = yy;
        } else if (f.mode == EPI_CHEB_FIRST) {
            const double v0 = f.vprev[o];
            const double v1 = ya * yy - yb * v0;
            f.vout[o] = v1;
            f.acc[o] = 0.5 * f.scal[8] * v0 + f.scal[9] * v1;
            if (f.dv) f.dv[o] = yy;
        } else {
            const double vp = 2.0 * (ya * yy - yb * f.vprev[o]) - f.vprev2[o];
            f.vout[o] = vp;
            f.acc[o] += f.scal[8 + f.p] * vp;
        }
    }
}

void launch_block_epi(const Ctx &c, const EpiArgs &f, hipStream_t s)
{
    hipLaunchKernelGGL(k_block_epi, dim3((c.N + 15) / 16), dim3(64 * EPI_W), 0, s, c.N, c.n3,
                       c.nk4, (c.nk + 15) / 16 * 16, c.eph, c.tkm, c.ypart, f, c.gate);
}

}  // namespace rpy
