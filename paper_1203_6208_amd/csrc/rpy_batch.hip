// rpy_batch.hip -- many independent periodic boxes of uneven size advanced
// together (the ensembles behind the averages of section "Testing and
// verification" of arXiv:1203.6208): every stage of the Brownian-dynamics
// step -- wrap, springs, real-space tiles, products with the reciprocal sum,
// Chebyshev coefficients, noise, Euler update -- is one launch over all
// boxes, and a whole step can be replayed as one HIP graph.
//
// Layout: box b owns the global beads [TBB tile0_b, TBB (tile0_b + nbt_b)),
// i.e. every box is padded to whole bead tiles of TBB beads, so the box of a
// bead is tile_box[bead / TBB].  Padding beads have zero forces, noise and
// vector entries and are never moved.  Stored real-space tiles of all boxes
// form one list (box, I, J) with I <= J inside the box; a product writes the
// per-tile partials into box-local slots part[K][j][row] (K < nbt_b) so that
// a row sums only the tile columns of its own box.  All boxes share alpha L
// and M, hence the same integer wave vectors; the weights 2 m(k) are per box.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <vector>

#include "rpy_internal.h"

namespace rpy {

constexpr int BRC = 2;                     // vector slots of the batched products
constexpr int BSCAL = 8 + MAX_NCHEB;       // per-box scalar block (as Ctx::scal)

struct BoxDev {
    int N, nchains, bpc, nbt;   // beads, chains, beads per chain, bead tiles
    int tile0;                  // first global bead tile
    int pad0, pad1, pad2;
    double L;
    PairConst pc;
};

// ---------------------------------------------------------------- per bead
template <int TBB>
__global__ void k_bwrap(int G, int nm1, const int *__restrict__ tile_box,
                        const BoxDev *__restrict__ boxes, const double *__restrict__ pos,
                        double *__restrict__ rt, double *__restrict__ sfr,
                        double2 *__restrict__ etab, int *__restrict__ flags)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    const BoxDev &d = boxes[tile_box[g / TBB]];
    const bool real = g - d.tile0 * TBB < d.N;
    bool bad = false;
    for (int i = 0; i < 3; ++i) {
        double r = real ? pos[3 * (size_t)g + i] : 0.0;
        if (!isfinite(r)) {
            bad = true;
            r = 0.0;
        }
        double s = r / d.L;
        s = s - floor(s);
        rt[3 * (size_t)g + i] = d.L * s;
        sfr[3 * (size_t)g + i] = s;
        double2 *tab = etab + (size_t)(3 * g + i) * nm1;
        for (int j = 0; j < nm1; ++j) {
            double sn, cs;
            sincospi(2.0 * j * s, &sn, &cs);
            tab[j] = make_double2(cs, sn);
        }
    }
    if (bad) atomicOr(flags, 1);
}

template <int TBB>
__global__ void k_bsprings(int G, const int *__restrict__ tile_box,
                           const BoxDev *__restrict__ boxes, const double *__restrict__ pos,
                           double *__restrict__ F)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    const BoxDev &d = boxes[tile_box[g / TBB]];
    const int loc = g - d.tile0 * TBB;
    const int b = loc % d.bpc;
    for (int i = 0; i < 3; ++i) {
        double f = 0.0;
        if (loc < d.N) {
            if (b + 1 < d.bpc) f += pos[3 * (size_t)(g + 1) + i] - pos[3 * (size_t)g + i];
            if (b > 0) f -= pos[3 * (size_t)g + i] - pos[3 * (size_t)(g - 1) + i];
        }
        F[3 * (size_t)g + i] = f;
    }
}

// Gaussian noise with the mapping of k_noise over the padded element index
// (block e/4, counter (e/4, step lo, step hi, 0x52505942), key (seed lo,
// seed hi), Box-Muller); padding elements are zero.  The step is read from
// the device counter so that graph replays draw fresh noise.
template <int TBB>
__global__ void k_bnoise(int G3, const int *__restrict__ tile_box,
                         const BoxDev *__restrict__ boxes, uint64_t seed,
                         const unsigned long long *__restrict__ stepc, double sdt,
                         double *__restrict__ out)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (4 * q >= G3) return;
    const uint64_t step = *stepc;
    const uint4 x = philox10(make_uint4((uint32_t)q, (uint32_t)step, (uint32_t)(step >> 32),
                                        0x52505942u),
                             make_uint2((uint32_t)seed, (uint32_t)(seed >> 32)));
    const double k = 1.0 / 4294967296.0;
    const double u0 = ((double)x.x + 0.5) * k, u1 = ((double)x.y + 0.5) * k;
    const double u2 = ((double)x.z + 0.5) * k, u3 = ((double)x.w + 0.5) * k;
    const double rho0 = sqrt(-2.0 * log(u0)), rho1 = sqrt(-2.0 * log(u2));
    double s1, c1, s3, c3;
    sincospi(2.0 * u1, &s1, &c1);
    sincospi(2.0 * u3, &s3, &c3);
    const double z[4] = {rho0 * c1, rho0 * s1, rho1 * c3, rho1 * s3};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int e = 4 * q + j;
        if (e >= G3) break;
        const int g = e / 3;
        const BoxDev &d = boxes[tile_box[g / TBB]];
        out[e] = (g - d.tile0 * TBB < d.N) ? z[j] * sdt : 0.0;
    }
}

template <int TBB>
__global__ void k_beuler(int G3, const int *__restrict__ tile_box,
                         const BoxDev *__restrict__ boxes, double *__restrict__ pos, double dt4,
                         const double *__restrict__ ud, const double *__restrict__ ds)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= G3) return;
    const int g = e / 3;
    const BoxDev &d = boxes[tile_box[g / TBB]];
    if (g - d.tile0 * TBB < d.N) pos[e] = pos[e] + dt4 * ud[e] + ds[e] / 1.4142135623730951;
}

// One lane: counter += 1 (a vector store from lane 0).
__global__ void k_bstep_inc(unsigned long long *stepc)
{
    if (threadIdx.x == 0) stepc[0] = stepc[0] + 1ull;
}

__global__ void k_bstep_set(unsigned long long *stepc, unsigned long long v)
{
    if (threadIdx.x == 0) stepc[0] = v;
}

// ------------------------------------------------------------- real space
// One workgroup per stored tile (box, I, J); as k_build_tiles with the box's
// pair constants and TBB-bead tiles, written as packed planes
// tile[i][c][j] (6 TBB^2 values, c = xx, xy, xz, yy, yz, zz: each 3 x 3
// bead-pair block is symmetric), FP64 and, with LOWP, FP32.
// Three waves per SIMD (189 VGPRs allow two): 4.72 against 5.09 ms for the
// 256-box ensemble.
template <int TBB, int LOWP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_bbuild(const int4 *__restrict__ stor,
                                                const BoxDev *__restrict__ boxes,
                                                const double *__restrict__ rt,
                                                double *__restrict__ d64, float *__restrict__ d32)
{
    constexpr int TSB = 3 * TBB;
    constexpr int STEP = 256 / TBB;
    __shared__ double sI[TSB], sJ[TSB];
    const int t = blockIdx.x;
    const int4 e = stor[t];
    const BoxDev &d = boxes[e.x];
    const int I = e.y, J = e.z;
    const int tid = threadIdx.x;
    const size_t gI = (size_t)(d.tile0 + I) * TBB, gJ = (size_t)(d.tile0 + J) * TBB;
    for (int q = tid; q < TSB; q += blockDim.x) {
        sI[q] = rt[3 * gI + q];
        sJ[q] = rt[3 * gJ + q];
    }
    __syncthreads();
    const int bj = tid % TBB, bi0 = tid / TBB;
    const int mu = J * TBB + bj;
    for (int s = 0; s < TBB / STEP; ++s) {
        const int bi = bi0 + STEP * s;
        const int nu = I * TBB + bi;
        double b[6] = {0, 0, 0, 0, 0, 0};
        if (nu < d.N && mu < d.N)
            pair_block(sI[3 * bi] - sJ[3 * bj], sI[3 * bi + 1] - sJ[3 * bj + 1],
                       sI[3 * bi + 2] - sJ[3 * bj + 2], nu == mu, d.pc, b);
        const size_t o6 = (size_t)t * 6 * TBB * TBB + (size_t)bi * 6 * TBB + bj;
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            d64[o6 + (size_t)e * TBB] = b[e];
            if (LOWP) d32[o6 + (size_t)e * TBB] = (float)b[e];
        }
    }
}

// ------------------------------------------------------------------ product
// Packed tiles: a bead row i of a tile holds 6 planes of TBB values.  Lane q
// (0..15) of a 16-lane row group owns NE = TBB/16 bead columns of every
// plane and reads them with one or two 16-byte (8-byte for FP32 32-bead
// tiles) non-temporal loads, contiguous across the row group.
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));
// A tile load: non-temporal (streamed past the caches) or, with CACHED, an
// ordinary load that allocates in the L2 and the Infinity Cache.
template <bool CACHED, typename V> __device__ inline V tload(const V *p)
{
    if constexpr (CACHED) return *p;
    else return __builtin_nontemporal_load(p);
}
template <typename T, int TBB> struct BLd;
template <> struct BLd<double, 64> {
    static constexpr int NE = 4;
    struct raw_t {
        d2v u, v;
    };
    __device__ static int col(int q, int e) { return 32 * (e >> 1) + 2 * q + (e & 1); }
    template <bool CACHED> __device__ static raw_t raw(const double *row, int q)
    {
        return {tload<CACHED>(reinterpret_cast<const d2v *>(row + 2 * q)),
                tload<CACHED>(reinterpret_cast<const d2v *>(row + 32 + 2 * q))};
    }
    __device__ static double at(const raw_t &r, int e)
    {
        return e == 0 ? r.u.x : e == 1 ? r.u.y : e == 2 ? r.v.x : r.v.y;
    }
};
template <> struct BLd<double, 32> {
    static constexpr int NE = 2;
    typedef d2v raw_t;
    __device__ static int col(int q, int e) { return 2 * q + e; }
    template <bool CACHED> __device__ static raw_t raw(const double *row, int q)
    {
        return tload<CACHED>(reinterpret_cast<const d2v *>(row + 2 * q));
    }
    __device__ static double at(const raw_t &u, int e) { return e == 0 ? u.x : u.y; }
};
template <> struct BLd<float, 64> {
    static constexpr int NE = 4;
    typedef f4v raw_t;
    __device__ static int col(int q, int e) { return 4 * q + e; }
    template <bool CACHED> __device__ static raw_t raw(const float *row, int q)
    {
        return tload<CACHED>(reinterpret_cast<const f4v *>(row + 4 * q));
    }
    __device__ static double at(const raw_t &u, int e) { return u[e]; }
};
template <> struct BLd<float, 32> {
    static constexpr int NE = 2;
    typedef f2v raw_t;
    __device__ static int col(int q, int e) { return 2 * q + e; }
    template <bool CACHED> __device__ static raw_t raw(const float *row, int q)
    {
        return tload<CACHED>(reinterpret_cast<const f2v *>(row + 2 * q));
    }
    __device__ static double at(const raw_t &u, int e) { return u[e]; }
};

// Structure-factor workgroups per bead tile: each stages the tile's phase
// tables once, so one workgroup walking all wave vectors reads them once
// (256 FP32 boxes: 6735 -> 6876 box-steps per second against one per block
// of 256 wave vectors; 6628 with two).
constexpr int BSF_SPLIT = 1;

// nsf structure-factor workgroups (spread over the launch, see below): the
// partials of one bead tile (chunk) for the wave vectors k = kb 256 + lane,
// stepping by nsplit 256 (kb < nsplit), one thread per k at a time:
//   sfpart[chunk][6 j + c][k] = sum over the chunk's real beads of
//   {cos, sin}(k.r) v_c.
// The other workgroups: one stored packed tile each, as the single-box FP64
// product (4 waves; a 16-lane row group per bead row; each lane owns the
// NE bead columns of BLd; FP64 accumulation for both tile types).
template <int TBB, typename T, int M, bool CACHED>
__global__ __launch_bounds__(256) void k_bsymv(int G3, int nsf, int sfr, int nsplit, int nk, int nm1,
                                               const int *__restrict__ tile_box,
                                               const BoxDev *__restrict__ boxes,
                                               const int4 *__restrict__ stor,
                                               const KVec *__restrict__ kvec,
                                               const double2 *__restrict__ etab,
                                               double *__restrict__ sfpart,
                                               const T *__restrict__ tiles,
                                               const double *__restrict__ v,
                                               double *__restrict__ part)
{
    constexpr int TSB = 3 * TBB;
    constexpr int NE = BLd<T, TBB>::NE;   // bead columns per lane
    extern __shared__ double smem[];
    // workgroup i is structure-factor workgroup i / sfr when i is a multiple
    // of sfr below nsf * sfr, else tile i - (structure-factor workgroups
    // before it): the structure factors are spread over the launch so that
    // their arithmetic overlaps the streaming of the tiles
    const int bid = blockIdx.x;
    const int nsf_before = min(nsf, bid / sfr + 1);
    if (bid % sfr == 0 && bid / sfr < nsf) {
        const int sfb = bid / sfr;
        const int chunk = sfb / nsplit, kb = sfb % nsplit;
        const BoxDev &d = boxes[tile_box[chunk]];
        const int loc0 = (chunk - d.tile0) * TBB;
        const int nb = max(0, min(TBB, d.N - loc0));
        const size_t g0 = (size_t)chunk * TBB;
        double2 *stab = reinterpret_cast<double2 *>(smem);      // [TBB][3 nm1]
        double *sv = smem + 2 * TBB * 3 * nm1;                   // [TBB][M][3]
        for (int q = threadIdx.x; q < nb * 3 * nm1; q += blockDim.x) stab[q] = etab[g0 * 3 * nm1 + q];
        for (int q = threadIdx.x; q < nb * 3 * M; q += blockDim.x) {
            const int bl = q / (3 * M), r = q % (3 * M), j = r / 3, c = r % 3;
            sv[q] = v[(size_t)j * G3 + 3 * (g0 + bl) + c];
        }
        __syncthreads();
        for (int k = kb * blockDim.x + threadIdx.x; k < nk; k += nsplit * blockDim.x) {
            const KVec kv = kvec[k];
            double acc[M][6];
#pragma unroll
            for (int j = 0; j < M; ++j)
#pragma unroll
                for (int c = 0; c < 6; ++c) acc[j][c] = 0.0;
            for (int bl = 0; bl < nb; ++bl) {
                const double2 *tab = stab + bl * 3 * nm1;
                double2 ex = tab[kv.nx];
                double2 ey = tab[nm1 + (kv.ny < 0 ? -kv.ny : kv.ny)];
                double2 ez = tab[2 * nm1 + (kv.nz < 0 ? -kv.nz : kv.nz)];
                if (kv.ny < 0) ey.y = -ey.y;
                if (kv.nz < 0) ez.y = -ez.y;
                const double xr = ex.x * ey.x - ex.y * ey.y, xi = ex.x * ey.y + ex.y * ey.x;
                const double cs = xr * ez.x - xi * ez.y, sn = xr * ez.y + xi * ez.x;
#pragma unroll
                for (int j = 0; j < M; ++j)
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const double x = sv[bl * 3 * M + 3 * j + c];
                        acc[j][c] += cs * x;
                        acc[j][3 + c] += sn * x;
                    }
            }
            double *o = sfpart + (size_t)chunk * 6 * BRC * nk + k;
#pragma unroll
            for (int j = 0; j < M; ++j)
#pragma unroll
                for (int c = 0; c < 6; ++c) o[(size_t)(6 * j + c) * nk] = acc[j][c];
        }
        return;
    }
    double(*sx)[TSB] = reinterpret_cast<double(*)[TSB]>(smem);                    // [M][TSB]
    double(*scol)[M][TSB] = reinterpret_cast<double(*)[M][TSB]>(smem + M * TSB);  // [4][M][TSB]
    const int t = bid - nsf_before;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane >> 4, q = lane & 15;
    // The tile's address needs only t: the first bead row's loads go out
    // before the vector loads, which wait on the tile table and the box
    // record.  With one vector the loop then loads each next row while the
    // current one is used (three waves per SIMD instead of four; 256 FP32
    // boxes: 6531 -> 6655 box-steps per second).  Two tiles per workgroup,
    // the second one's first row loaded during the first one's column
    // combine, lost (5899, and 6263 without that load).
    const T *tile = tiles + (size_t)t * 6 * TBB * TBB;
    constexpr bool PF = M == 1;
    typename BLd<T, TBB>::raw_t rw[TBB / 16][6];
#pragma unroll
    for (int c = 0; c < 6; ++c)
        rw[0][c] = BLd<T, TBB>::template raw<CACHED>(tile + (size_t)(4 * w + g) * 6 * TBB + c * TBB, q);
    const int4 e = stor[t];
    const BoxDev &d = boxes[e.x];
    const int I = e.y, J = e.z;
    const size_t rowI = 3 * (size_t)(d.tile0 + I) * TBB, rowJ = 3 * (size_t)(d.tile0 + J) * TBB;
    // the vector loads of x_I (for LDS) and x_J (registers) all go out
    // before the first LDS store, which waits for them (256 threads)
    constexpr int NSX = (M * TSB + 255) / 256;
    double sxv[NSX];
#pragma unroll
    for (int u = 0; u < NSX; ++u) {
        const int z = threadIdx.x + 256 * u;
        sxv[u] = z < M * TSB ? v[(size_t)(z / TSB) * G3 + rowI + z % TSB] : 0.0;
    }
    double xj[M][NE][3];
#pragma unroll
    for (int j = 0; j < M; ++j)
#pragma unroll
        for (int c = 0; c < NE; ++c)
#pragma unroll
            for (int x = 0; x < 3; ++x)
                xj[j][c][x] = v[(size_t)j * G3 + rowJ + 3 * BLd<T, TBB>::col(q, c) + x];
#pragma unroll
    for (int u = 0; u < NSX; ++u) {
        const int z = threadIdx.x + 256 * u;
        if (z < M * TSB) sx[z / TSB][z % TSB] = sxv[u];
    }
    double cacc[M][NE][3];
#pragma unroll
    for (int j = 0; j < M; ++j)
#pragma unroll
        for (int c = 0; c < NE; ++c) cacc[j][c][0] = cacc[j][c][1] = cacc[j][c][2] = 0.0;
    __syncthreads();
    const bool offd = I != J;
#pragma unroll
    for (int it = 0; it < TBB / 16; ++it) {
        const int i = 16 * it + 4 * w + g;
        if constexpr (PF) {
            if (it + 1 < TBB / 16) {
#pragma unroll
                for (int c = 0; c < 6; ++c)
                    rw[it + 1][c] = BLd<T, TBB>::template raw<CACHED>(
                        tile + (size_t)(i + 16) * 6 * TBB + c * TBB, q);
            }
            // compiler-only barrier: keeps the next row's loads ahead of this
            // row's arithmetic
            __asm__ volatile("" ::: "memory");
        } else if (it > 0) {
#pragma unroll
            for (int c = 0; c < 6; ++c)
                rw[it][c] = BLd<T, TBB>::template raw<CACHED>(tile + (size_t)i * 6 * TBB + c * TBB, q);
        }
        // one bead column at a time: its six entries are widened where they
        // are used (fewer live registers than widening the whole row)
        double r[M][3], y[M][3];
#pragma unroll
        for (int j = 0; j < M; ++j)
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                r[j][x] = 0.0;
                y[j][x] = sx[j][3 * i + x];
            }
#pragma unroll
        for (int c = 0; c < NE; ++c) {
            double b[6];
#pragma unroll
            for (int p = 0; p < 6; ++p) b[p] = BLd<T, TBB>::at(rw[it][p], c);
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const double x0 = xj[j][c][0], x1 = xj[j][c][1], x2 = xj[j][c][2];
                r[j][0] += b[0] * x0 + b[1] * x1 + b[2] * x2;
                r[j][1] += b[1] * x0 + b[3] * x1 + b[4] * x2;
                r[j][2] += b[2] * x0 + b[4] * x1 + b[5] * x2;
                if (offd) {
                    cacc[j][c][0] += b[0] * y[j][0] + b[1] * y[j][1] + b[2] * y[j][2];
                    cacc[j][c][1] += b[1] * y[j][0] + b[3] * y[j][1] + b[4] * y[j][2];
                    cacc[j][c][2] += b[2] * y[j][0] + b[4] * y[j][1] + b[5] * y[j][2];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < M; ++j) {
            double r0 = r[j][0], r1 = r[j][1], r2 = r[j][2];
#pragma unroll
            for (int o = 8; o >= 1; o >>= 1) {
                r0 += __shfl_xor(r0, o, 16);
                r1 += __shfl_xor(r1, o, 16);
                r2 += __shfl_xor(r2, o, 16);
            }
            if (q < 3)
                part[((size_t)J * BRC + j) * G3 + rowI + 3 * i + q] = q == 0 ? r0 : q == 1 ? r1 : r2;
        }
    }
    if (!offd) return;
#pragma unroll
    for (int j = 0; j < M; ++j)
#pragma unroll
        for (int c = 0; c < NE; ++c)
#pragma unroll
            for (int x = 0; x < 3; ++x) {
                double s = cacc[j][c][x];
                s += __shfl_xor(s, 16);
                s += __shfl_xor(s, 32);
                if (g == 0) scol[w][j][3 * BLd<T, TBB>::col(q, c) + x] = s;
            }
    __syncthreads();
    for (int z = threadIdx.x; z < M * TSB; z += blockDim.x) {
        const int j = z / TSB, ci = z % TSB;
        const double s = ((scol[0][j][ci] + scol[1][j][ci]) + scol[2][j][ci]) + scol[3][j][ci];
        part[((size_t)I * BRC + j) * G3 + rowJ + ci] = s;
    }
}

// Chunk sum and T_k = 2 m(k) (I - khat khat) (C_k or S_k) of every box: one
// thread per (k, vector j, half), grid (k blocks of 64, 2 M, box).  The
// chunks of the box are summed in ascending order (loads coalesced over k).
// Output tk[box][j][k][6] = (T^C_k, T^S_k).
__global__ __launch_bounds__(64) void k_bsf_reduce(int nk, const BoxDev *__restrict__ boxes,
                                                   const KCoef *__restrict__ kcoef,
                                                   const double *__restrict__ sfpart,
                                                   double *__restrict__ tk)
{
    const BoxDev &d = boxes[blockIdx.z];
    const int k = blockIdx.x * 64 + threadIdx.x;
    if (k >= nk) return;
    const int j = blockIdx.y >> 1, half = blockIdx.y & 1;
    const size_t cst = (size_t)6 * BRC * nk;
    const double *o = sfpart + (size_t)d.tile0 * cst + (size_t)(6 * j + 3 * half) * nk + k;
    double t0 = 0.0, t1 = 0.0, t2 = 0.0;
    const int nb = d.nbt;
    int ch = 0;
    for (; ch + 4 <= nb; ch += 4) {
        double a[4][3];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double *p = o + (size_t)(ch + q) * cst;
            a[q][0] = p[0];
            a[q][1] = p[nk];
            a[q][2] = p[2 * (size_t)nk];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            t0 += a[q][0];
            t1 += a[q][1];
            t2 += a[q][2];
        }
    }
    for (; ch < nb; ++ch) {
        const double *p = o + (size_t)ch * cst;
        t0 += p[0];
        t1 += p[nk];
        t2 += p[2 * (size_t)nk];
    }
    const KCoef kc = kcoef[(size_t)blockIdx.z * nk + k];
    const double h = kc.hx * t0 + kc.hy * t1 + kc.hz * t2;
    double *out = tk + (((size_t)blockIdx.z * BRC + j) * nk + k) * 6 + 3 * half;
    out[0] = kc.w * (t0 - kc.hx * h);
    out[1] = kc.w * (t1 - kc.hy * h);
    out[2] = kc.w * (t2 - kc.hz * h);
}

// Back-projection + partial sum + epilogue of one bead tile (TBB beads of
// one box), 256 threads: S = 256 / TBB slices per bead.  Slice u sums the
// box's tile-column slots K = u, u + S, ... and the wave vectors
// [u nk / S, (u + 1) nk / S).  The wave vectors are walked as runs of
// consecutive n_z at fixed (n_x, n_y) (runs[r] = (n_x, n_y, first n_z, first
// k), runs[nruns].w = nk; krun[k] = run of k); the phase of bead l is
// e^{i 2 pi n.s} = ex[n_x] ey[n_y] ez[n_z] from its wrap tables (negative
// components conjugate) at the slice's first wave vector of a run, then
// advanced by e^{i 2 pi s_z} per step in n_z.  Slices are combined in
// ascending order.  STAGE: the box's T_k are copied to LDS (else read from
// global memory; with 64-bead tiles every wave is one slice, so the wave
// vector index is wave-uniform and T_k come through scalar loads straight
// into the multiply-adds' operands).  Every global load of the prologue (partial slots, tables,
// T_k) is issued before the first wait (the table pointers are not
// __restrict__ so that the compiler keeps the loads where they are written).  Padding beads get zero outputs;
// recurrence scalars are per box.
constexpr int EPI_SLOTS = 8;    // partial slots per slice held in registers
constexpr int EPI_TAB = 6;      // table entries (double2) per thread and round
constexpr int EPI_TK = 8;       // T_k entries (double2) per thread and round
// Wave vectors per pass of the back-projection loop (256 FP32 boxes with
// scalar T_k loads: 7108-7148 box-steps per second, 7085 with 2, 6926 with
// 1, 7033 with 8).
constexpr int BEPI_KU = 4;

template <int TBB, int M, bool STAGE>
__global__ __launch_bounds__(256) void k_bepi(int G3, int nk, int nm1, int nruns,
                                              const int *__restrict__ tile_box,
                                              const BoxDev *__restrict__ boxes,
                                              const int4 *__restrict__ runs,
                                              const int *__restrict__ krun,
                                              const double2 *etab,
                                              const double *__restrict__ part,
                                              const double *__restrict__ tk, EpiArgs f,
                                              const double *__restrict__ scal_all)
{
    constexpr int S = 256 / TBB;
    extern __shared__ double sm[];
    const int tile = blockIdx.x;
    const int b = tile_box[tile];
    const BoxDev &d = boxes[b];
    const double *scal = scal_all ? scal_all + (size_t)b * BSCAL : nullptr;
    const double *tkb = tk + (size_t)b * BRC * nk * 6;   // [j][k][6] of this box
    // LDS: phase tables [3 nm1][TBB] (double2) + 1 slack entry, runs
    // [nruns + 1] (int4), then the staged T_k [M][nk][6] + 1 slack double2.
    // Loads past the end are clamped and their copies land in the slack
    // entries, so that loads and LDS writes stay unconditional (and batched).
    const int ntab = 3 * nm1 * TBB;
    double2 *tab = reinterpret_cast<double2 *>(sm);
    int4 *srun = reinterpret_cast<int4 *>(sm + 2 * (ntab + 1));
    double *stk = sm + 2 * (ntab + 1) + 2 * (nruns + 1);
    const int l = threadIdx.x % TBB;
    // one slice per wave with 64-bead tiles: the slice and everything derived
    // from it are wave-uniform, so T_k come through scalar loads
    const int u = TBB == 64 ? __builtin_amdgcn_readfirstlane((int)threadIdx.x / TBB) : (int)threadIdx.x / TBB;
    const int g = tile * TBB + l;
    const bool live = (tile - d.tile0) * TBB + l < d.N;
    const int nbt = d.nbt;
    // partial slots K = u + S i (i < EPI_SLOTS per round), clamped addresses
    double y[M][3];
#pragma unroll
    for (int j = 0; j < M; ++j) y[j][0] = y[j][1] = y[j][2] = 0.0;
    for (int K0 = u; K0 < nbt; K0 += S * EPI_SLOTS) {
        double pv[EPI_SLOTS][M][3];
#pragma unroll
        for (int i = 0; i < EPI_SLOTS; ++i) {
            const int K = min(K0 + S * i, nbt - 1);
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const double *pp = part + ((size_t)K * BRC + j) * G3 + 3 * (size_t)g;
                pv[i][j][0] = pp[0];
                pv[i][j][1] = pp[1];
                pv[i][j][2] = pp[2];
            }
        }
#pragma unroll
        for (int i = 0; i < EPI_SLOTS; ++i)
#pragma unroll
            for (int j = 0; j < M; ++j)
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    y[j][c] += K0 + S * i < nbt ? pv[i][j][c] : 0.0;
    }
    // phase tables of the tile's beads
    for (int q0 = 0; q0 < ntab; q0 += 256 * EPI_TAB) {
        double2 tv[EPI_TAB];
#pragma unroll
        for (int i = 0; i < EPI_TAB; ++i) {
            const int q = min(q0 + 256 * i + (int)threadIdx.x, ntab - 1);
            const int ql = q % TBB, rj = q / TBB;   // rj = axis * nm1 + j
            tv[i] = etab[(size_t)(tile * TBB + ql) * 3 * nm1 + rj];
        }
#pragma unroll
        for (int i = 0; i < EPI_TAB; ++i) tab[min(q0 + 256 * i + (int)threadIdx.x, ntab)] = tv[i];
    }
    for (int q = threadIdx.x; q <= nruns; q += 256) srun[q] = runs[q];
    if (STAGE) {
        const int ntk = nk * 3 * M;   // double2 entries of T_k for j < M
        const double2 *src = reinterpret_cast<const double2 *>(tkb);
        double2 *dst = reinterpret_cast<double2 *>(stk);
        for (int q0 = 0; q0 < ntk; q0 += 256 * EPI_TK) {
            double2 tv[EPI_TK];
#pragma unroll
            for (int i = 0; i < EPI_TK; ++i)
                tv[i] = src[min(q0 + 256 * i + (int)threadIdx.x, ntk - 1)];
#pragma unroll
            for (int i = 0; i < EPI_TK; ++i) dst[min(q0 + 256 * i + (int)threadIdx.x, ntk)] = tv[i];
        }
    }
    const int klo = (int)((long)u * nk / S), khi = (int)((long)(u + 1) * nk / S);
    const int r0 = klo < khi ? krun[klo] : 0;
    __syncthreads();
    const double *tks = STAGE ? stk : tkb;
    if (live) {
        const double2 *tx = tab + l, *ty = tab + nm1 * TBB + l, *tz = tab + 2 * nm1 * TBB + l;
        const double2 ez1 = nm1 > 1 ? tz[TBB] : make_double2(1.0, 0.0);   // e^{i 2 pi s_z}
        int k = klo;
        for (int r = r0; k < khi; ++r) {
            int4 R = srun[r];
            int kend = min(khi, srun[r + 1].w);
            if (TBB == 64) {
                R.x = __builtin_amdgcn_readfirstlane(R.x);
                R.y = __builtin_amdgcn_readfirstlane(R.y);
                R.z = __builtin_amdgcn_readfirstlane(R.z);
                R.w = __builtin_amdgcn_readfirstlane(R.w);
                kend = __builtin_amdgcn_readfirstlane(kend);
            }
            const double2 ex = tx[R.x * TBB];
            double2 ey = ty[(R.y < 0 ? -R.y : R.y) * TBB];
            if (R.y < 0) ey.y = -ey.y;
            const double xr = ex.x * ey.x - ex.y * ey.y, xi = ex.x * ey.y + ex.y * ey.x;
            // the phase at the slice's first wave vector of this run from the
            // tables, then one factor e^{i 2 pi s_z} per step in n_z
            const int nz0 = R.z + (k - R.w);
            double2 ez = tz[(nz0 < 0 ? -nz0 : nz0) * TBB];
            if (nz0 < 0) ez.y = -ez.y;
            double cs = xr * ez.x - xi * ez.y, sn = xr * ez.y + xi * ez.x;
            // BEPI_KU wave vectors per pass with their T_k reads issued
            // together, then the rest one at a time
            for (; k + BEPI_KU <= kend; k += BEPI_KU) {
                double tt[BEPI_KU][M][6];
#pragma unroll
                for (int q = 0; q < BEPI_KU; ++q)
#pragma unroll
                    for (int j = 0; j < M; ++j)
#pragma unroll
                        for (int c = 0; c < 6; ++c) tt[q][j][c] = tks[((size_t)j * nk + k + q) * 6 + c];
#pragma unroll
                for (int q = 0; q < BEPI_KU; ++q) {
#pragma unroll
                    for (int j = 0; j < M; ++j)
#pragma unroll
                        for (int c = 0; c < 3; ++c)
                            y[j][c] = fma(sn, tt[q][j][3 + c], fma(cs, tt[q][j][c], y[j][c]));
                    const double c2 = cs * ez1.x - sn * ez1.y;
                    sn = cs * ez1.y + sn * ez1.x;
                    cs = c2;
                }
            }
            for (; k < kend; ++k) {
#pragma unroll
                for (int j = 0; j < M; ++j) {
                    const double *tt = tks + ((size_t)j * nk + k) * 6;
#pragma unroll
                    for (int c = 0; c < 3; ++c) y[j][c] = fma(sn, tt[3 + c], fma(cs, tt[c], y[j][c]));
                }
                const double c2 = cs * ez1.x - sn * ez1.y;
                sn = cs * ez1.y + sn * ez1.x;
                cs = c2;
            }
        }
    }
    __syncthreads();   // tables and staged T_k are reused below
    double *red = sm;  // [S][3 M][TBB]
#pragma unroll
    for (int j = 0; j < M; ++j)
#pragma unroll
        for (int c = 0; c < 3; ++c) red[(u * 3 * M + 3 * j + c) * TBB + l] = y[j][c];
    __syncthreads();
    const double ya = scal ? scal[2] : 0.0, yb = scal ? scal[3] : 0.0;
    const int nreal = d.N - (tile - d.tile0) * TBB;   // real beads of this tile (may exceed TBB)
    for (int q = threadIdx.x; q < 3 * TBB * M; q += 256) {
        const int j = q / (3 * TBB), qq = q % (3 * TBB);
        const int bl = qq / 3, c = qq % 3;
        const size_t o = (size_t)j * G3 + 3 * (size_t)tile * TBB + qq;
        if (bl >= nreal) {   // padding bead: zero outputs
            f.vout[o] = 0.0;
            if (f.mode != EPI_APPLY) f.acc[o] = 0.0;
            if (f.mode == EPI_CHEB_FIRST && f.dv) f.dv[o] = 0.0;
            continue;
        }
        double yy = 0.0;
#pragma unroll
        for (int w = 0; w < S; ++w) yy += red[(w * 3 * M + 3 * j + c) * TBB + bl];
        if (f.mode == EPI_APPLY) {
            f.vout[o] = yy;
        } else if (f.mode == EPI_CHEB_FIRST) {
            const double v0 = f.vprev[o];
            const double v1 = ya * yy - yb * v0;
            f.vout[o] = v1;
            f.acc[o] = 0.5 * scal[8] * v0 + scal[9] * v1;
            if (f.dv) f.dv[o] = yy;
        } else {
            const double vp = 2.0 * (ya * yy - yb * f.vprev[o]) - f.vprev2[o];
            f.vout[o] = vp;
            f.acc[o] += scal[8 + f.p] * vp;
        }
    }
}

// Chebyshev interval and coefficients of every box (one workgroup per box),
// as k_cheb_coeffs: the paper's rule from du = D.U+ of the box, or the
// explicit interval.
__global__ __launch_bounds__(1024) void k_bcoeffs(int n, int rule, double C, double dmin,
                                                  double dmax, const BoxDev *__restrict__ boxes,
                                                  const double *__restrict__ du,
                                                  double *__restrict__ scal_all, int TBB)
{
    __shared__ double red[1024];
    __shared__ double bounds[2];
    const BoxDev &d = boxes[blockIdx.x];
    double *scal = scal_all + (size_t)blockIdx.x * BSCAL;
    const int tid = threadIdx.x;
    if (rule == RPY_BOUNDS_PAPER) {
        const int n3 = 3 * d.N;
        const double *x = du + 3 * (size_t)d.tile0 * TBB;
        double s0 = 0.0;
        for (int i = tid; i < n3; i += 1024) s0 += x[i];
        red[tid] = s0;
        __syncthreads();
        for (int h = 512; h > 0; h >>= 1) {
            if (tid < h) red[tid] += red[tid + h];
            __syncthreads();
        }
        if (tid == 0) {
            const double lf = red[0] / n3;
            const double np6 = pow((double)d.N, 0.6);
            const double lmax = 0.35 * np6 * lf;
            bounds[0] = lmax / (C * np6);
            bounds[1] = lmax;
        }
    } else if (tid == 0) {
        bounds[0] = dmin;
        bounds[1] = dmax;
    }
    __syncthreads();
    const double lo = bounds[0], hi = bounds[1];
    const double h = 0.5 * (hi - lo), mid = 0.5 * (hi + lo);
    const int lane = tid & 63, w = tid >> 6;
    for (int p = w; p < n; p += 16) {
        double s = 0.0;
        for (int j = 1 + lane; j <= n; j += 64) {
            const double uu = (j - 0.5) / n;
            s += sqrt(h * cospi(uu) + mid) * cospi(p * uu);
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
        if (lane == 0) scal[8 + p] = 2.0 * s / n;
    }
    if (tid == 0) {
        scal[0] = lo;
        scal[1] = hi;
        scal[2] = 2.0 / (hi - lo);
        scal[3] = (hi + lo) / (hi - lo);
    }
}

// U+ in the padded layout: 1 on the beads of a box, 0 on padding.
template <int TBB>
__global__ void k_bones(int G3, const int *__restrict__ tile_box,
                        const BoxDev *__restrict__ boxes, double *__restrict__ u)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= G3) return;
    const int g = e / 3;
    const BoxDev &d = boxes[tile_box[g / TBB]];
    u[e] = (g - d.tile0 * TBB < d.N) ? 1.0 : 0.0;
}

// E_f of every box (one workgroup per box), as k_sqrt_error over the box's
// 3 N entries.
__global__ __launch_bounds__(256) void k_bsqrt_error(const BoxDev *__restrict__ boxes, int TBB,
                                                     const double *__restrict__ dw,
                                                     const double *__restrict__ ddw,
                                                     const double *__restrict__ ds,
                                                     double *__restrict__ e_f)
{
    __shared__ double r1[256], r2[256];
    const BoxDev &d = boxes[blockIdx.x];
    const size_t o0 = 3 * (size_t)d.tile0 * TBB;
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < 3 * d.N; i += blockDim.x) {
        a += ds[o0 + i] * ds[o0 + i];
        b += dw[o0 + i] * ddw[o0 + i];
    }
    r1[threadIdx.x] = a;
    r2[threadIdx.x] = b;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            r1[threadIdx.x] += r1[threadIdx.x + h];
            r2[threadIdx.x] += r2[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) e_f[blockIdx.x] = sqrt(fabs(r1[0] - r2[0]) / r2[0]);
}

// Per-chain R_e^2 and R_g^2 of every box; chains listed as (box, chain).
template <int TBB>
__global__ void k_bobs(int nch, const int2 *__restrict__ chains,
                       const BoxDev *__restrict__ boxes, const double *__restrict__ pos,
                       double *__restrict__ re2, double *__restrict__ rg2)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nch) return;
    const int2 bc = chains[q];
    const BoxDev &d = boxes[bc.x];
    const int bpc = d.bpc;
    const double *x = pos + 3 * ((size_t)d.tile0 * TBB + (size_t)bc.y * bpc);
    double cm[3] = {0, 0, 0};
    for (int b = 0; b < bpc; ++b)
        for (int i = 0; i < 3; ++i) cm[i] += x[3 * b + i];
    for (int i = 0; i < 3; ++i) cm[i] /= bpc;
    double gg = 0.0;
    for (int b = 0; b < bpc; ++b)
        for (int i = 0; i < 3; ++i) {
            const double dd = x[3 * b + i] - cm[i];
            gg += dd * dd;
        }
    double ee = 0.0;
    for (int i = 0; i < 3; ++i) {
        const double dd = x[3 * (bpc - 1) + i] - x[i];
        ee += dd * dd;
    }
    re2[q] = ee;
    rg2[q] = gg / bpc;
}

}  // namespace rpy

// =================================================================== C ABI
using namespace rpy;

struct rpy_batch {
    int nbox = 0, tbb = 64, lowp = RPY_PREC_F64;
    int sf_front = 0, tile_cached = 0;   // product variant (rpy_batch_set_variant)
    int G = 0, ntb = 0, nstor = 0, maxnbt = 0, nchain = 0;
    int nk = 0, nmax = 0;
    std::vector<int64_t> bead0;   // padded bead offsets of the boxes (nbox + 1)
    std::vector<int> nbeads;      // beads of each box
    BoxDev *boxes = nullptr;
    int *tile_box = nullptr;      // [ntb]
    int4 *stor = nullptr;         // [nstor] (box, I, J, 0)
    int2 *chains = nullptr;       // [nchain] (box, chain)
    KVec *kvec = nullptr;         // [nk], shared by all boxes
    int nruns = 0;
    int4 *runs = nullptr;         // [nruns + 1] runs of consecutive n_z (n_x, n_y, n_z0, k0)
    int *krun = nullptr;          // [nk] run of each wave vector
    KCoef *kcoef = nullptr;       // [nbox][nk]
    double *rt = nullptr, *sfr = nullptr;   // [G][3]
    double2 *etab = nullptr;      // [G][3][nmax + 1]
    double *d64 = nullptr;        // [nstor][6 TBB^2] packed planes
    float *d32 = nullptr;
    double *part = nullptr;       // [maxnbt][BRC][3G]
    double *sfpart = nullptr;     // [ntb][6 BRC][nk]
    double *tk = nullptr;         // [nbox][BRC][nk][6]
    double *scal = nullptr;       // [nbox][BSCAL]
    double *work = nullptr;
    double *FU = nullptr;         // [2][3G]: forces, U+
    double *Y = nullptr;          // [2][3G]: D.F, D.U+
    double *dW = nullptr, *dS = nullptr, *ddw = nullptr;
    double *Bv[2] = {nullptr, nullptr};
    int *flags = nullptr;
    unsigned long long *stepc = nullptr;
    hipStream_t cs = nullptr;     // capture stream
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    double *gpos = nullptr;       // what the captured step was recorded for
    bd_params gbp{};
    uint64_t gseed = 0;
};

#define BHIP(x)                                          \
    do {                                                 \
        hipError_t e_ = (x);                             \
        if (e_ != hipSuccess) return hip_error(e_, #x);  \
    } while (0)

template <typename T> static int balloc(T **p, size_t n)
{
    if (n == 0) n = 1;
    if (hipMalloc((void **)p, n * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        char m[96];
        snprintf(m, sizeof m, "hipMalloc(%zu bytes) failed", n * sizeof(T));
        set_error(m);
        return RPY_ENOMEM;
    }
    return RPY_OK;
}

static int blaunch_ok(const char *what)
{
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? RPY_OK : hip_error(e, what);
}

extern "C" void rpy_batch_destroy(rpy_batch *b)
{
    if (!b) return;
    (void)hipDeviceSynchronize();
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cs) (void)hipStreamDestroy(b->cs);
    void *bufs[] = {b->boxes, b->tile_box, b->stor, b->chains, b->kvec, b->runs, b->krun,
                    b->kcoef, b->rt,
                    b->sfr, b->etab, b->d64, b->d32, b->part, b->sfpart, b->tk, b->scal,
                    b->work, b->flags, b->stepc};
    for (void *p : bufs)
        if (p) (void)hipFree(p);
    delete b;
}

extern "C" int rpy_batch_create(rpy_batch **out, const rpy_params *bp, int nbox, int lowp,
                                int tile_beads)
{
    if (!out) return RPY_EINVAL;
    *out = nullptr;
    if (!bp || nbox < 1 || nbox > 65535) {
        set_error("need 1..65535 boxes");
        return RPY_EINVAL;
    }
    if (lowp != RPY_PREC_F64 && lowp != RPY_PREC_F32) {
        set_error("batched lowp must be RPY_PREC_F64 or RPY_PREC_F32");
        return RPY_EINVAL;
    }
    if (tile_beads != 32 && tile_beads != 64) {
        set_error("tile_beads must be 32 or 64");
        return RPY_EINVAL;
    }
    int n2max = -1;
    for (int i = 0; i < nbox; ++i) {
        int n2 = 0;
        const int rc = validate_params(&bp[i], &n2);
        if (rc) return rc;
        if (n2max >= 0 && n2 != n2max) {
            set_error("all boxes need the same wave-vector set (equal floor((k_c L / 2 pi)^2))");
            return RPY_EINVAL;
        }
        n2max = n2;
    }
    rpy_batch *b = new (std::nothrow) rpy_batch();
    if (!b) return RPY_ENOMEM;
    b->nbox = nbox;
    b->tbb = tile_beads;
    b->lowp = lowp;
    const int TBB = tile_beads;
    int nmax = (int)floor(sqrt((double)n2max));
    while ((nmax + 1) * (nmax + 1) <= n2max) ++nmax;
    while (nmax * nmax > n2max) --nmax;
    b->nmax = nmax;

    std::vector<BoxDev> hb(nbox);
    std::vector<int> tbox;
    std::vector<int4> stor;
    std::vector<int2> chains;
    b->bead0.assign(nbox + 1, 0);
    b->nbeads.assign(nbox, 0);
    for (int i = 0; i < nbox; ++i) {
        BoxDev &d = hb[i];
        memset(&d, 0, sizeof d);
        d.N = bp[i].n_beads;
        d.nchains = bp[i].n_chains;
        d.bpc = bp[i].beads_per_chain;
        d.nbt = (d.N + TBB - 1) / TBB;
        d.tile0 = (int)tbox.size();
        d.L = bp[i].box_l;
        d.pc = make_pair_const(bp[i].box_l, bp[i].a, bp[i].alpha, bp[i].r_c);
        for (int t = 0; t < d.nbt; ++t) tbox.push_back(i);
        for (int I = 0; I < d.nbt; ++I)
            for (int J = I; J < d.nbt; ++J) stor.push_back(make_int4(i, I, J, 0));
        for (int ch = 0; ch < d.nchains; ++ch) chains.push_back(make_int2(i, ch));
        b->maxnbt = d.nbt > b->maxnbt ? d.nbt : b->maxnbt;
        b->bead0[i] = (int64_t)d.tile0 * TBB;
        b->nbeads[i] = d.N;
        if ((int64_t)tbox.size() * TBB * 3 > 0x7fffffffLL) {
            set_error("batch too large: 3 x padded beads must fit in int32");
            delete b;
            return RPY_EINVAL;
        }
    }
    b->ntb = (int)tbox.size();
    b->G = b->ntb * TBB;
    b->bead0[nbox] = b->G;
    b->nstor = (int)stor.size();
    b->nchain = (int)chains.size();

    // half-space wave vectors (one integer set) and per-box weights
    std::vector<KVec> kv;
    for (int nx = 0; nx <= nmax; ++nx)
        for (int ny = -nmax; ny <= nmax; ++ny)
            for (int nz = -nmax; nz <= nmax; ++nz) {
                const int n2 = nx * nx + ny * ny + nz * nz;
                if (n2 == 0 || n2 > n2max) continue;
                if (nx == 0 && (ny < 0 || (ny == 0 && nz < 0))) continue;
                kv.push_back(KVec{nx, ny, nz, 0});
            }
    b->nk = (int)kv.size();
    std::vector<int4> runs;
    std::vector<int> krun(b->nk);
    for (int k = 0; k < b->nk; ++k) {
        if (k == 0 || kv[k].nx != kv[k - 1].nx || kv[k].ny != kv[k - 1].ny ||
            kv[k].nz != kv[k - 1].nz + 1)
            runs.push_back(make_int4(kv[k].nx, kv[k].ny, kv[k].nz, k));
        krun[k] = (int)runs.size() - 1;
    }
    b->nruns = (int)runs.size();
    runs.push_back(make_int4(0, 0, 0, b->nk));   // sentinel: end of the last run
    std::vector<KCoef> kc((size_t)nbox * b->nk);
    for (int i = 0; i < nbox; ++i) {
        const double L = bp[i].box_l, a = bp[i].a, al2 = bp[i].alpha * bp[i].alpha;
        const double vol = L * L * L;
        for (int k = 0; k < b->nk; ++k) {
            const double kx = 2.0 * M_PI * kv[k].nx / L, ky = 2.0 * M_PI * kv[k].ny / L,
                         kz = 2.0 * M_PI * kv[k].nz / L;
            const double k2 = kx * kx + ky * ky + kz * kz, kn = sqrt(k2);
            const double mk = (a - a * a * a * k2 / 3.0) *
                              (1.0 + k2 / (4.0 * al2) + k2 * k2 / (8.0 * al2 * al2)) *
                              (6.0 * M_PI / (k2 * vol)) * exp(-k2 / (4.0 * al2));
            kc[(size_t)i * b->nk + k] = KCoef{2.0 * mk, kx / kn, ky / kn, kz / kn};
        }
    }

    const size_t G3 = 3 * (size_t)b->G;
    const size_t te = (size_t)b->nstor * 6 * TBB * TBB;
    int rc;
    if ((rc = balloc(&b->boxes, nbox)) || (rc = balloc(&b->tile_box, b->ntb)) ||
        (rc = balloc(&b->stor, b->nstor)) || (rc = balloc(&b->chains, b->nchain)) ||
        (rc = balloc(&b->kvec, b->nk)) || (rc = balloc(&b->runs, runs.size())) ||
        (rc = balloc(&b->krun, b->nk)) || (rc = balloc(&b->kcoef, kc.size())) ||
        (rc = balloc(&b->rt, G3)) || (rc = balloc(&b->sfr, G3)) ||
        (rc = balloc(&b->etab, G3 * (nmax + 1))) || (rc = balloc(&b->d64, te)) ||
        (lowp == RPY_PREC_F32 && (rc = balloc(&b->d32, te))) ||
        (rc = balloc(&b->part, (size_t)b->maxnbt * BRC * G3)) ||
        (rc = balloc(&b->sfpart, (size_t)b->ntb * 6 * BRC * b->nk)) ||
        (rc = balloc(&b->tk, (size_t)nbox * b->nk * BRC * 6)) ||
        (rc = balloc(&b->scal, (size_t)nbox * BSCAL)) || (rc = balloc(&b->work, 9 * G3)) ||
        (rc = balloc(&b->flags, 4)) || (rc = balloc(&b->stepc, 1))) {
        rpy_batch_destroy(b);
        return rc;
    }
    double *w = b->work;
    b->FU = w; w += 2 * G3;
    b->Y = w; w += 2 * G3;
    b->dW = w; w += G3;
    b->dS = w; w += G3;
    b->ddw = w; w += G3;
    b->Bv[0] = w; w += G3;
    b->Bv[1] = w; w += G3;
    hipError_t e;
    if ((e = hipMemcpy(b->boxes, hb.data(), nbox * sizeof(BoxDev), hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(b->tile_box, tbox.data(), tbox.size() * sizeof(int),
                       hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(b->stor, stor.data(), stor.size() * sizeof(int4), hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(b->chains, chains.data(), chains.size() * sizeof(int2),
                       hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(b->kvec, kv.data(), kv.size() * sizeof(KVec), hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(b->runs, runs.data(), runs.size() * sizeof(int4), hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(b->krun, krun.data(), krun.size() * sizeof(int), hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(b->kcoef, kc.data(), kc.size() * sizeof(KCoef), hipMemcpyHostToDevice)) ||
        (e = hipMemset(b->flags, 0, 4 * sizeof(int))) ||
        (e = hipMemset(b->work, 0, 9 * G3 * sizeof(double))) ||
        (e = hipMemset(b->stepc, 0, sizeof(unsigned long long))) ||
        (e = hipStreamCreateWithFlags(&b->cs, hipStreamNonBlocking))) {
        rc = hip_error(e, "rpy_batch_create upload");
        rpy_batch_destroy(b);
        return rc;
    }
    const unsigned gb = (unsigned)((G3 + 255) / 256);
    if (TBB == 32)
        hipLaunchKernelGGL(k_bones<32>, dim3(gb), dim3(256), 0, 0, (int)G3, b->tile_box, b->boxes,
                           b->FU + G3);
    else
        hipLaunchKernelGGL(k_bones<64>, dim3(gb), dim3(256), 0, 0, (int)G3, b->tile_box, b->boxes,
                           b->FU + G3);
    if ((e = hipDeviceSynchronize()) != hipSuccess) {
        rc = hip_error(e, "rpy_batch_create sync");
        rpy_batch_destroy(b);
        return rc;
    }
    *out = b;
    return RPY_OK;
}

extern "C" int64_t rpy_batch_padded_beads(const rpy_batch *b) { return b ? b->G : -1; }

extern "C" int rpy_batch_offsets(const rpy_batch *b, int64_t *bead0)
{
    if (!b || !bead0) return RPY_EINVAL;
    memcpy(bead0, b->bead0.data(), sizeof(int64_t) * (b->nbox + 1));
    return RPY_OK;
}

static inline hipStream_t BS(void *s) { return reinterpret_cast<hipStream_t>(s); }

// ------------------------------------------------------------ stage sequence
template <int TBB> static void bwrap_build(rpy_batch *b, const double *pos, hipStream_t s)
{
    const unsigned gg = (unsigned)((b->G + 255) / 256);
    hipLaunchKernelGGL(k_bwrap<TBB>, dim3(gg), dim3(256), 0, s, b->G, b->nmax + 1, b->tile_box,
                       b->boxes, pos, b->rt, b->sfr, b->etab, b->flags);
    if (b->lowp == RPY_PREC_F32)
        hipLaunchKernelGGL((k_bbuild<TBB, 1>), dim3(b->nstor), dim3(256), 0, s, b->stor, b->boxes,
                           b->rt, b->d64, b->d32);
    else
        hipLaunchKernelGGL((k_bbuild<TBB, 0>), dim3(b->nstor), dim3(256), 0, s, b->stor, b->boxes,
                           b->rt, b->d64, b->d32);
}

template <int TBB, typename T, int M>
static void bsymv(rpy_batch *b, const T *tiles, const double *v, hipStream_t s)
{
    const int nm1 = b->nmax + 1, nsplit = BSF_SPLIT < (b->nk + 255) / 256 ? BSF_SPLIT : (b->nk + 255) / 256;
    const int nsf = b->ntb * nsplit;
    const size_t sm_sf = (size_t)(2 * TBB * 3 * nm1 + TBB * 3 * M) * sizeof(double);
    const size_t sm_t = (size_t)5 * M * 3 * TBB * sizeof(double);
    const int total = nsf + b->nstor;
    // spread: one structure-factor workgroup every sfr; front: the first nsf
    const int sfr = b->sf_front ? 1 : (total / nsf > 1 ? total / nsf : 1);
    const size_t lds = sm_sf > sm_t ? sm_sf : sm_t;
    if (b->tile_cached)
        hipLaunchKernelGGL((k_bsymv<TBB, T, M, true>), dim3(total), dim3(256), lds, s, 3 * b->G,
                           nsf, sfr, nsplit, b->nk, nm1, b->tile_box, b->boxes, b->stor, b->kvec,
                           b->etab, b->sfpart, tiles, v, b->part);
    else
        hipLaunchKernelGGL((k_bsymv<TBB, T, M, false>), dim3(total), dim3(256), lds, s, 3 * b->G,
                           nsf, sfr, nsplit, b->nk, nm1, b->tile_box, b->boxes, b->stor, b->kvec,
                           b->etab, b->sfpart, tiles, v, b->part);
}

// y = D.v for m = 1 or 2 vectors in the padded layout, epilogue f.
template <int TBB>
static void bproduct(rpy_batch *b, const double *v, int m, int prec, const EpiArgs &f,
                     const double *scal, hipStream_t s)
{
    if (prec == RPY_PREC_F32) {
        if (m == 2) bsymv<TBB, float, 2>(b, b->d32, v, s);
        else bsymv<TBB, float, 1>(b, b->d32, v, s);
    } else {
        if (m == 2) bsymv<TBB, double, 2>(b, b->d64, v, s);
        else bsymv<TBB, double, 1>(b, b->d64, v, s);
    }
    hipLaunchKernelGGL(k_bsf_reduce, dim3((b->nk + 63) / 64, 2 * m, b->nbox), dim3(64), 0, s,
                       b->nk, b->boxes, b->kcoef, b->sfpart, b->tk);
    // LDS: phase tables and runs, plus, for 32-bead tiles, the box's T_k
    // when they fit in 64 KiB together; the region is reused for the slice
    // sums.  64-bead tiles read T_k with scalar loads instead: half the LDS,
    // twice the resident workgroups (256 FP32 boxes: 6863 -> 7060
    // box-steps per second)
    const int nm1 = b->nmax + 1;
    const size_t tabb = (size_t)(3 * nm1 * TBB + 1) * sizeof(double2) +
                        (size_t)(b->nruns + 1) * sizeof(int4);
    const size_t red = (size_t)3 * m * 256 * sizeof(double);
    const size_t stk = (size_t)b->nk * 6 * m * sizeof(double) + sizeof(double2);
    // staging T_k costs occupancy: with two vectors (82 KB of LDS at 618
    // wave vectors) the back-projection took 762 against 531 us unstaged
    const bool stage = TBB != 64 && tabb + stk <= 65536;
    size_t lds = tabb + (stage ? stk : 0);
    lds = lds > red ? lds : red;
    const dim3 ge((unsigned)b->ntb);
#define RPY_BEPI(MM, ST)                                                                      \
    hipLaunchKernelGGL((k_bepi<TBB, MM, ST>), ge, dim3(256), lds, s, 3 * b->G, b->nk, nm1,    \
                       b->nruns, b->tile_box, b->boxes, b->runs, b->krun, b->etab, b->part,  \
                       b->tk, f, scal)
    if (m == 2) {
        if (stage) RPY_BEPI(2, true);
        else RPY_BEPI(2, false);
    } else {
        if (stage) RPY_BEPI(1, true);
        else RPY_BEPI(1, false);
    }
#undef RPY_BEPI
}

// Chebyshev interval + coefficients of every box and the recurrence on dw.
template <int TBB>
static void bcheb(rpy_batch *b, const double *dw, double *out, int n_cheb, int rule, double C,
                  double dmin, double dmax, const double *du, int prec, hipStream_t s)
{
    hipLaunchKernelGGL(k_bcoeffs, dim3(b->nbox), dim3(1024), 0, s, n_cheb, rule, C, dmin, dmax,
                       b->boxes, du, b->scal, TBB);
    for (int p = 1; p < n_cheb; ++p) {
        EpiArgs f{};
        f.m = 1;
        f.p = p;
        f.acc = out;
        if (p == 1) {
            f.mode = EPI_CHEB_FIRST;
            f.vprev = dw;
            f.vout = b->Bv[1];
            f.dv = b->ddw;
        } else {
            f.mode = EPI_CHEB_NEXT;
            f.vprev = b->Bv[(p - 1) % 2];
            f.vprev2 = p == 2 ? dw : b->Bv[p % 2];
            f.vout = b->Bv[p % 2];
        }
        bproduct<TBB>(b, f.vprev, 1, prec, f, b->scal, s);
    }
}

// One Brownian-dynamics step of every box; the noise step index is read from
// the device counter b->stepc.
template <int TBB>
static void bstep_body(rpy_batch *b, double *pos, const bd_params *bp, uint64_t seed,
                       hipStream_t s)
{
    const int G3 = 3 * b->G;
    bwrap_build<TBB>(b, pos, s);
    hipLaunchKernelGGL(k_bsprings<TBB>, dim3((b->G + 255) / 256), dim3(256), 0, s, b->G,
                       b->tile_box, b->boxes, pos, b->FU);
    EpiArgs f{};
    f.mode = EPI_APPLY;
    f.vout = b->Y;
    const bool paper = bp->bounds_rule == RPY_BOUNDS_PAPER;
    f.m = paper ? 2 : 1;   // [F, U+] in one pass when the interval comes from D.U+
    bproduct<TBB>(b, b->FU, f.m, RPY_PREC_F64, f, nullptr, s);
    hipLaunchKernelGGL(k_bnoise<TBB>, dim3((unsigned)(((G3 + 3) / 4 + 255) / 256)), dim3(256), 0,
                       s, G3, b->tile_box, b->boxes, seed, b->stepc, sqrt(bp->dt), b->dW);
    bcheb<TBB>(b, b->dW, b->dS, bp->n_cheb, bp->bounds_rule, bp->bounds_C, bp->d_min, bp->d_max,
               b->Y + G3, bp->prec, s);
    hipLaunchKernelGGL(k_beuler<TBB>, dim3((G3 + 255) / 256), dim3(256), 0, s, G3, b->tile_box,
                       b->boxes, pos, bp->dt / 4.0, b->Y, b->dS);
}

static bool bprec_ok(const rpy_batch *b, int prec)
{
    return prec == RPY_PREC_F64 || (prec == RPY_PREC_F32 && b->lowp == RPY_PREC_F32);
}

static int bcheck_bd(const rpy_batch *b, const bd_params *bp)
{
    if (!(bp->dt > 0) || !isfinite(bp->dt) || bp->n_cheb < 2 || bp->n_cheb > MAX_NCHEB ||
        !bprec_ok(b, bp->prec))
        return RPY_EINVAL;
    if (bp->ev_zstar != 0.0) {
        set_error("batched boxes run without excluded volume (ev_zstar must be 0)");
        return RPY_EINVAL;
    }
    if (bp->tol > 0) {
        set_error("batched boxes take a fixed Chebyshev order (tol must be <= 0)");
        return RPY_EINVAL;
    }
    if (bp->bounds_rule == RPY_BOUNDS_EXPLICIT)
        return (bp->d_min > 0 && bp->d_max > bp->d_min && isfinite(bp->d_max)) ? RPY_OK
                                                                             : RPY_EINVAL;
    if (bp->bounds_rule == RPY_BOUNDS_PAPER) return bp->bounds_C > 0 ? RPY_OK : RPY_EINVAL;
    return RPY_EINVAL;
}

// ------------------------------------------------------------------ entries
extern "C" int rpy_batch_build(rpy_batch *b, const double *pos, void *stream)
{
    if (!b || !pos) return RPY_EINVAL;
    if (b->tbb == 32) bwrap_build<32>(b, pos, BS(stream));
    else bwrap_build<64>(b, pos, BS(stream));
    return blaunch_ok("rpy_batch_build");
}

extern "C" int rpy_batch_apply(rpy_batch *b, const double *v, double *out, int m, int prec,
                               void *stream)
{
    if (!b || !v || !out || m < 1 || m > BRC || !bprec_ok(b, prec)) return RPY_EINVAL;
    EpiArgs f{};
    f.mode = EPI_APPLY;
    f.m = m;
    f.vout = out;
    if (b->tbb == 32) bproduct<32>(b, v, m, prec, f, nullptr, BS(stream));
    else bproduct<64>(b, v, m, prec, f, nullptr, BS(stream));
    return blaunch_ok("rpy_batch_apply");
}

extern "C" int rpy_batch_chebyshev(rpy_batch *b, const double *dw, double *out, int n_cheb,
                                   int bounds_rule, double C, double d_min, double d_max, int prec,
                                   double *e_f, double *bounds, void *stream)
{
    if (!b || !dw || !out || n_cheb < 2 || n_cheb > MAX_NCHEB || !bprec_ok(b, prec))
        return RPY_EINVAL;
    if (bounds_rule == RPY_BOUNDS_EXPLICIT) {
        if (!(d_min > 0) || !(d_max > d_min) || !isfinite(d_max)) return RPY_EINVAL;
    } else if (bounds_rule != RPY_BOUNDS_PAPER || !(C > 0)) {
        return RPY_EINVAL;
    }
    hipStream_t s = BS(stream);
    const int G3 = 3 * b->G;
    const double *du = nullptr;
    if (bounds_rule == RPY_BOUNDS_PAPER) {
        EpiArgs f{};
        f.mode = EPI_APPLY;
        f.m = 1;
        f.vout = b->Y + G3;
        if (b->tbb == 32) bproduct<32>(b, b->FU + G3, 1, RPY_PREC_F64, f, nullptr, s);
        else bproduct<64>(b, b->FU + G3, 1, RPY_PREC_F64, f, nullptr, s);
        du = b->Y + G3;
    }
    if (b->tbb == 32) bcheb<32>(b, dw, out, n_cheb, bounds_rule, C, d_min, d_max, du, prec, s);
    else bcheb<64>(b, dw, out, n_cheb, bounds_rule, C, d_min, d_max, du, prec, s);
    if (e_f)
        hipLaunchKernelGGL(k_bsqrt_error, dim3(b->nbox), dim3(256), 0, s, b->boxes, b->tbb, dw,
                           b->ddw, out, e_f);
    if (bounds)
        BHIP(hipMemcpy2DAsync(bounds, 2 * sizeof(double), b->scal, BSCAL * sizeof(double),
                              2 * sizeof(double), b->nbox, hipMemcpyDeviceToDevice, s));
    return blaunch_ok("rpy_batch_chebyshev");
}

extern "C" int rpy_batch_step(rpy_batch *b, double *pos, const bd_params *bp, uint64_t seed,
                              uint64_t step, double *drift, double *noise, double *e_f,
                              void *stream)
{
    if (!b || !pos || !bp) return RPY_EINVAL;
    int rc = bcheck_bd(b, bp);
    if (rc) return rc;
    hipStream_t s = BS(stream);
    const size_t G3 = 3 * (size_t)b->G;
    hipLaunchKernelGGL(k_bstep_set, dim3(1), dim3(64), 0, s, b->stepc, (unsigned long long)step);
    if (b->tbb == 32) bstep_body<32>(b, pos, bp, seed, s);
    else bstep_body<64>(b, pos, bp, seed, s);
    if (e_f)
        hipLaunchKernelGGL(k_bsqrt_error, dim3(b->nbox), dim3(256), 0, s, b->boxes, b->tbb, b->dW,
                           b->ddw, b->dS, e_f);
    if (drift) launch_copy(drift, b->Y, G3, s);
    if (noise) launch_copy(noise, b->dS, G3, s);
    return blaunch_ok("rpy_batch_step");
}

// n_steps steps as replays of one captured step.  The graph is recorded on
// the first call and again whenever pos, *bp or seed differ from the recorded
// ones; it holds kernel nodes only (the step counter is advanced by a kernel).
extern "C" int rpy_batch_run(rpy_batch *b, double *pos, const bd_params *bp, uint64_t seed,
                             uint64_t step0, int n_steps, void *stream)
{
    if (!b || !pos || !bp || n_steps < 0) return RPY_EINVAL;
    int rc = bcheck_bd(b, bp);
    if (rc) return rc;
    hipStream_t s = BS(stream);
    const bool same = b->gexec && b->gpos == pos && b->gseed == seed &&
                      memcmp(&b->gbp, bp, sizeof(bd_params)) == 0;
    if (!same) {
        if (b->gexec) {
            BHIP(hipGraphExecDestroy(b->gexec));
            b->gexec = nullptr;
        }
        if (b->graph) {
            BHIP(hipGraphDestroy(b->graph));
            b->graph = nullptr;
        }
        BHIP(hipStreamBeginCapture(b->cs, hipStreamCaptureModeThreadLocal));
        if (b->tbb == 32) bstep_body<32>(b, pos, bp, seed, b->cs);
        else bstep_body<64>(b, pos, bp, seed, b->cs);
        hipLaunchKernelGGL(k_bstep_inc, dim3(1), dim3(64), 0, b->cs, b->stepc);
        const hipError_t le = hipGetLastError();
        hipGraph_t g = nullptr;
        const hipError_t ce = hipStreamEndCapture(b->cs, &g);
        if (le != hipSuccess || ce != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_error(le != hipSuccess ? le : ce, "rpy_batch_run capture");
        }
        b->graph = g;
        BHIP(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
        b->gpos = pos;
        b->gbp = *bp;
        b->gseed = seed;
    }
    hipLaunchKernelGGL(k_bstep_set, dim3(1), dim3(64), 0, s, b->stepc, (unsigned long long)step0);
    rc = blaunch_ok("rpy_batch_run");
    if (rc) return rc;
    for (int i = 0; i < n_steps; ++i) BHIP(hipGraphLaunch(b->gexec, s));
    return RPY_OK;
}

static void bgraph_drop(rpy_batch *b)
{
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
}

extern "C" int rpy_batch_set_variant(rpy_batch *b, int sf_place, int tile_loads)
{
    if (!b || (sf_place != RPY_SF_SPREAD && sf_place != RPY_SF_FRONT) ||
        (tile_loads != RPY_LOADS_STREAM && tile_loads != RPY_LOADS_CACHED))
        return RPY_EINVAL;
    const int front = sf_place == RPY_SF_FRONT, cached = tile_loads == RPY_LOADS_CACHED;
    if (front != b->sf_front || cached != b->tile_cached) {
        BHIP(hipDeviceSynchronize());   // a replay in flight keeps its own variant
        bgraph_drop(b);
        b->sf_front = front;
        b->tile_cached = cached;
    }
    return RPY_OK;
}

extern "C" int64_t rpy_batch_graph_nodes(const rpy_batch *b)
{
    if (!b || !b->graph) return -1;
    size_t n = 0;
    if (hipGraphGetNodes(b->graph, nullptr, &n) != hipSuccess) return -1;
    return (int64_t)n;
}

extern "C" int rpy_batch_observables(rpy_batch *b, const double *pos, double *re2, double *rg2,
                                     void *stream)
{
    if (!b || !pos || !re2 || !rg2) return RPY_EINVAL;
    const dim3 g((unsigned)((b->nchain + 255) / 256));
    if (b->tbb == 32)
        hipLaunchKernelGGL(k_bobs<32>, g, dim3(256), 0, BS(stream), b->nchain, b->chains,
                           b->boxes, pos, re2, rg2);
    else
        hipLaunchKernelGGL(k_bobs<64>, g, dim3(256), 0, BS(stream), b->nchain, b->chains,
                           b->boxes, pos, re2, rg2);
    return blaunch_ok("rpy_batch_observables");
}

extern "C" int rpy_batch_status(rpy_batch *b, void *stream)
{
    if (!b) return RPY_EINVAL;
    BHIP(hipStreamSynchronize(BS(stream)));
    int fl = 0;
    BHIP(hipMemcpy(&fl, b->flags, sizeof fl, hipMemcpyDeviceToHost));
    if (fl) {
        BHIP(hipMemset(b->flags, 0, sizeof(int)));
        set_error("non-finite position");
        return RPY_ENONFINITE;
    }
    return RPY_OK;
}
