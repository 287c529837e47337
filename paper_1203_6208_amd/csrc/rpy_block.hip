// rpy_block.hip -- the block product Y = D.V for 5 to 16 vectors at once, as
// used by the Chebyshev recurrence (arXiv:1203.6208, eq. cheb1-cheb3: every
// term is one product of D with the current vectors), on the matrix cores.
//
//   1. k_pack_block: the vectors in the operand layouts below (the tile
//      product's element type, component-major; FP64 for the reciprocal sum).
//   2. k_block_tiles: the stored packed tiles (FP64, FP32 or BF16, the same
//      6 planes per bead row that every other product reads) times the
//      vectors on the matrix cores, accumulation in FP64 (FP64 tiles) or FP32
//      inside a tile, one partial per tile and tile column:
//      bpart[K][row][j].
//   3. k_block_sf + k_block_sf_reduce: structure factors S_k = sum_mu e^{i k.r_mu}
//      v_mu as an FP64 matrix-core product of the phase matrix (computed once
//      per set of positions by k_block_phases) with V, then the fixed-order
//      chunk sum and 2 m(k) (I - khat khat) (eq. DF, third term, evaluated
//      per product).  Extra workgroups of the same launch sum the tile
//      partials in slot order.
//   4. k_block_epi: the back-projection sum_k (cos, sin)(k.r_nu) T_k as an
//      FP64 matrix-core product, plus the summed tile partials, plus the
//      recurrence step.
// The reciprocal sum and the recurrence are FP64 throughout.
//
// Tile product.  A stored tile (I <= J) holds, for bead rows i and columns j
// of the two bead tiles, the six planes P_ab[i][j] (ab = xx, xy, xz, yy, yz,
// zz) of the symmetric 3 x 3 blocks.  With x_J[j][b] the vectors of the beads
// of J:
//   row product     y_I[i][a] += sum_j P_ab[i][j] x_J[j][b]   -> slot J
//   column product  y_J[j][b] += sum_i P_ab[i][j] x_I[i][a]   -> slot I (I < J)
// for every plane and, off the plane diagonal (a != b), for ab and ba alike.
// Each is a 64 x 64 plane times a 64 x 16 vector block: MFMA 16x16 blocks of
// 16 beads x 16 vectors, FP64 16x16x4 for FP64 tiles, FP32 16x16x4 for FP32
// tiles and BF16 16x16x32 (the vectors split into a hi + lo BF16 pair, so
// only D is rounded) for BF16 tiles.
#include <hip/hip_ext.h>

#include "rpy_internal.h"

namespace rpy {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));
typedef double d4v __attribute__((ext_vector_type(4)));
typedef uint32_t u4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

constexpr int SF_WAVES = 4;    // waves per structure-factor workgroup
constexpr int SF_U = 16;       // unrolled steps per block (quads per wave at N = 4000)
constexpr int SF_PF = 3;       // steps loaded ahead
constexpr int EPI_U = 10;      // the same for the back-projection (two blocks at 618 k)
constexpr int EPI_PF = 3;

__device__ inline uint16_t bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Packed vectors, zero for beads >= N and vectors >= m (npad = padded beads):
//   FP64, FP32: xs[c][bead][j]
//   BF16:       xh[c][j][bead] = bf16(x), xl[c][j][bead] = bf16(x - xh), xl
//               at xh + 3 npad 16 (a hi + lo pair: about 16 significant bits)
//   FP64:       vpk[r][j], r = 3 bead + c (the reciprocal sum's operand)
// so that a workgroup stages the 64 beads of a bead tile with contiguous
// loads, and 16 lanes read 16 vectors of one row together.  pack_entry writes
// one (bead, c, j) entry of both; k_pack_block packs a whole block (zeros
// included), and the Chebyshev epilogue packs its output for the next product.
__device__ inline void pack_entry(int prec, int npad, int bead, int c, int j, double x,
                                  void *__restrict__ xs, double *__restrict__ vpk)
{
    vpk[(size_t)(3 * bead + c) * BLOCK_RHS + j] = x;
    if (prec == RPY_PREC_BF16) {
        const size_t o = (size_t)(c * BLOCK_RHS + j) * npad + bead;
        uint16_t *xh = reinterpret_cast<uint16_t *>(xs);
        const uint16_t h = bf16_rne((float)x);
        const double hv = (double)__uint_as_float((uint32_t)h << 16);
        xh[o] = h;
        xh[(size_t)3 * npad * BLOCK_RHS + o] = bf16_rne((float)(x - hv));
    } else {
        const size_t o = ((size_t)c * npad + bead) * BLOCK_RHS + j;
        if (prec == RPY_PREC_F64) reinterpret_cast<double *>(xs)[o] = x;
        else reinterpret_cast<float *>(xs)[o] = (float)x;
    }
}

// One thread per packed entry (bead < npad, c, j < 16).
__global__ void k_pack_block(int N, int n3, int npad, int m, int prec,
                             const double *__restrict__ v, void *__restrict__ xs,
                             double *__restrict__ vpk, const int *__restrict__ gate)
{
    if (gate && *gate) return;   // a product past the settled adaptive order
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= 3 * npad * BLOCK_RHS) return;
    const int j = o & 15, r = o >> 4, bead = r / 3, c = r % 3;
    const double x = (j < m && bead < N) ? v[(size_t)j * n3 + r] : 0.0;
    pack_entry(prec, npad, bead, c, j, x, xs, vpk);
}

// Per element type: the lane's 16-byte loads of a plane row, the vector and
// accumulator types, the LDS row stride of a transposed plane (padded so
// that the 16 rows a read instruction touches spread over the banks), and
// the waves of a tile's workgroup: 8 for FP64 and FP32 (each contraction
// split in two halves, 2.0x and 1.1x faster than 4 waves at N = 4000, FP64
// 150.6 -> 129.7 us, FP32 69.0 -> 61.9 us), 4 for BF16 (the matrix cores are
// lightly loaded and the extra barriers cost more: 35.7 against 44.9 us).
//   A wave holds 16 bead rows i = 16 w + (lane % 16) of a plane; lane group
//   g = lane / 16 loads NLD pieces of EPL entries, the piece p covering the
//   columns col(p, g, e) = 4 EPL p + EPL g + e, e < EPL.  A matrix-core step
//   contracts over the 4 (FP64, FP32: one entry each) or 32 (BF16: EPL = 8
//   each) columns that the four lane groups hold for one (p, e) (BF16: one
//   p); the vector operand of lane (g, n) is x at the same column, vector n.
template <typename T> struct BK;
template <> struct BK<double> {
    typedef d2v ld_t;
    typedef double x_t;
    typedef d4v acc_t;
    typedef double part_t;
    static constexpr int EPL = 2, NLD = 8, PLD = 66, NWAVE = 8;
    // accumulator entry e of lane group g is row g + 4 e of the 16 x 16 block
    __device__ static int orow(int g, int e) { return g + 4 * e; }
};
template <> struct BK<float> {
    typedef f4v ld_t;
    typedef float x_t;
    typedef f4v acc_t;
    typedef float part_t;
    static constexpr int EPL = 4, NLD = 4, PLD = 68, NWAVE = 8;
    __device__ static int orow(int g, int e) { return 4 * g + e; }
};
template <> struct BK<uint16_t> {
    typedef u4v ld_t;
    typedef uint16_t x_t;
    typedef f4v acc_t;
    typedef float part_t;
    static constexpr int EPL = 8, NLD = 2, PLD = 72, NWAVE = 4;
    __device__ static int orow(int g, int e) { return 4 * g + e; }
};

__device__ inline int plane_a(int c) { return c < 3 ? 0 : (c < 5 ? 1 : 2); }
__device__ inline int plane_b(int c) { return c < 3 ? c : (c < 5 ? c - 2 : 2); }

__device__ inline d4v mfma(double a, double b, d4v c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4v mfma(float a, float b, f4v c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline f4v mfma(u4v a, u4v b, f4v c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8v, a),
                                                   __builtin_bit_cast(bf8v, b), c, 0, 0, 0);
}

// A wave's part of a plane stripe: NH loads of 16 bytes per lane, the
// pieces h NH .. (h + 1) NH - 1 (NH = NLD with 4 waves, NLD / 2 with 8).  The streamed operand is not declared
// __restrict__ and the ring lives in fixed registers (the caller's loop is
// unrolled): loads the compiler may treat as invariant get rematerialised at
// their use, which undoes the prefetch.
template <typename T> struct Stripe {
    typename BK<T>::ld_t v[BK<T>::NLD * 4 / BK<T>::NWAVE];
};

template <typename T, bool CACHED>
__device__ inline void load_stripe(const T *tiles, int t, int c, int row, int g, int h,
                                   Stripe<T> &s)
{
    typedef typename BK<T>::ld_t L;
    constexpr int NH = BK<T>::NLD * 4 / BK<T>::NWAVE;
    const T *p = tiles + (size_t)t * TILE6 + ((size_t)row * 6 + c) * TB + BK<T>::EPL * g +
                 4 * BK<T>::EPL * NH * h;
#pragma unroll
    for (int k = 0; k < NH; ++k) {
        const L *a = reinterpret_cast<const L *>(p + 4 * BK<T>::EPL * k);
        if constexpr (CACHED) s.v[k] = *a;
        else s.v[k] = __builtin_nontemporal_load(a);
    }
}

// LDS of a workgroup: the vectors of both bead tiles, and two buffers of one
// transposed plane, pb[col][row].
template <typename T> struct alignas(32) BlkLds {
    static constexpr int XN = 3 * TB * BLOCK_RHS;   // entries per bead tile (x 2 for BF16 hi/lo)
    static constexpr int XW = (sizeof(T) == 2 ? 2 : 1) * XN;
    typename BK<T>::x_t xj[XW], xi[XW];
    T pb[2][TB * BK<T>::PLD];
};

// Workgroup b (4 or 8 waves) takes the stored tiles b, b + gridDim.x, ... (a
// persistent loop, so that the plane loads run ahead across tiles).  Wave w
// (row group r = w % 4, half h = w / 4) owns the bead rows 16 r .. 16 r + 15
// for the row product and the bead columns 16 r .. 16 r + 15 for the column
// product, and (with 8 waves) half of each contraction: the columns (row
// product) and rows (column product) of the pieces h NH .. (h + 1) NH - 1.
// Per plane it loads its part of the rows (two planes ahead), runs its part
// of the row product from registers, writes those rows transposed to LDS,
// and after one barrier runs its part of the column product.  With 8 waves
// the two halves are added at the end of a tile in a fixed order (h = 0 plus
// h = 1).  Diagonal tiles hold
// both (i, j) and (j, i) and take the row product only.  The partials of a
// tile go to bpart[K][row][j] (K = J, rows of I for the row product; K = I,
// rows of J for the column product), every (K, row) written by exactly one
// tile.
template <typename T, bool CACHED>
__global__ __launch_bounds__(64 * BK<T>::NWAVE) void k_block_tiles(int ntiles, int npad, int n3pad,
                                                     const int2 *__restrict__ tile_ij,
                                                     const T *tiles,
                                                     const typename BK<T>::x_t *__restrict__ xs,
                                                     typename BK<T>::part_t *__restrict__ bpart,
                                                     const int *__restrict__ gate)
{
    typedef BK<T> K;
    typedef typename K::acc_t A;
    typedef typename K::x_t X;
    typedef typename K::part_t P;
    constexpr int EPL = K::EPL, NLD = K::NLD, PLD = K::PLD, NW = K::NWAVE, NH = NLD * 4 / NW;
    constexpr bool BF = sizeof(T) == 2;
    constexpr int XN = BlkLds<T>::XN;
    __shared__ BlkLds<T> L;
    static_assert(sizeof(BlkLds<T>) >= 4 * 64 * 6 * sizeof(A), "LDS too small for the halves");
    if (gate && *gate) return;   // a product past the settled adaptive order
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rg = w & 3, h = w >> 2;
    const int n = lane & 15, g = lane >> 4;
    const int row = 16 * rg + n;   // this lane's bead row of a plane stripe (column of P^T)
    const int step = gridDim.x;
    Stripe<T> ring[3];
    int t = blockIdx.x;
    if (t < ntiles) {
        load_stripe<T, CACHED>(tiles, t, 0, row, g, h, ring[0]);
        load_stripe<T, CACHED>(tiles, t, 1, row, g, h, ring[1]);
    }
    for (; t < ntiles; t += step) {
        const int2 ij = tile_ij[t];
        const int I = ij.x, J = ij.y;
        const bool offd = I != J;
        __syncthreads();   // the previous tile's readers of L are done
        // stage the vectors of J (row product) and I (column product)
        if constexpr (BF) {
            const X *xh = xs, *xl = xs + (size_t)3 * npad * BLOCK_RHS;
            for (int e = threadIdx.x; e < 2 * XN; e += 64 * NW) {
                const int hl = e / XN, r = e % XN, cj = r / TB, bead = r % TB;
                const size_t o = (size_t)cj * npad + bead;
                L.xj[e] = (hl ? xl : xh)[o + (size_t)J * TB];
                L.xi[e] = (hl ? xl : xh)[o + (size_t)I * TB];
            }
        } else {
            for (int e = threadIdx.x; e < XN; e += 64 * NW) {
                const int c = e / (TB * BLOCK_RHS), r = e % (TB * BLOCK_RHS);
                const size_t o = (size_t)c * npad * BLOCK_RHS + r;
                L.xj[e] = xs[o + (size_t)J * TB * BLOCK_RHS];
                L.xi[e] = xs[o + (size_t)I * TB * BLOCK_RHS];
            }
        }
        A dacc[3], tacc[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) dacc[a] = tacc[a] = A{};
        __syncthreads();
        const int tn = t + step;   // the tile whose first planes are loaded at the end
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            // two planes ahead; planes 4 and 5 fetch planes 0 and 1 of the next tile
            if (c + 2 < 6) load_stripe<T, CACHED>(tiles, t, c + 2, row, g, h, ring[(c + 2) % 3]);
            else if (tn < ntiles) load_stripe<T, CACHED>(tiles, tn, c - 4, row, g, h, ring[(c + 2) % 3]);
            __asm__ volatile("" ::: "memory");
            const Stripe<T> &st = ring[c % 3];
            const int a = plane_a(c), b = plane_b(c);
            // row product: A = P rows (this lane's row, columns col(p, g, e)),
            // B = x_J at those columns
#pragma unroll
            for (int pp = 0; pp < NH; ++pp) {
                const int p = NH * h + pp;
                if constexpr (BF) {
                    const int col0 = 4 * EPL * p + EPL * g;
                    const u4v av = st.v[pp];
                    const u4v xbh = *reinterpret_cast<const u4v *>(&L.xj[(b * 16 + n) * TB + col0]);
                    const u4v xbl = *reinterpret_cast<const u4v *>(&L.xj[XN + (b * 16 + n) * TB + col0]);
                    dacc[a] = mfma(av, xbh, dacc[a]);
                    dacc[a] = mfma(av, xbl, dacc[a]);
                    if (a != b) {
                        const u4v xah = *reinterpret_cast<const u4v *>(&L.xj[(a * 16 + n) * TB + col0]);
                        const u4v xal = *reinterpret_cast<const u4v *>(&L.xj[XN + (a * 16 + n) * TB + col0]);
                        dacc[b] = mfma(av, xah, dacc[b]);
                        dacc[b] = mfma(av, xal, dacc[b]);
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < EPL; ++e) {
                        const int col = 4 * EPL * p + EPL * g + e;
                        const X av = st.v[pp][e];
                        dacc[a] = mfma(av, L.xj[(b * TB + col) * 16 + n], dacc[a]);
                        if (a != b) dacc[b] = mfma(av, L.xj[(a * TB + col) * 16 + n], dacc[b]);
                    }
                }
            }
            if (offd) {
                // this wave's half rows -> LDS, transposed: pb[col][row]
                T *pb = L.pb[c & 1];
#pragma unroll
                for (int pp = 0; pp < NH; ++pp) {
                    const int p = NH * h + pp;
                    if constexpr (BF) {
                        const u4v av = st.v[pp];
#pragma unroll
                        for (int e = 0; e < 8; ++e) {
                            const uint32_t wd = av[e >> 1];
                            pb[(4 * EPL * p + EPL * g + e) * PLD + row] =
                                (uint16_t)((e & 1) ? (wd >> 16) : (wd & 0xFFFFu));
                        }
                    } else {
#pragma unroll
                        for (int e = 0; e < EPL; ++e)
                            pb[(4 * EPL * p + EPL * g + e) * PLD + row] = st.v[pp][e];
                    }
                }
            }
            __syncthreads();
            if (offd) {
                // column product: A = P^T rows (this lane's column, rows
                // col(p, g, e) of the plane), B = x_I at those rows
                const T *pr = L.pb[c & 1] + (size_t)row * PLD;
#pragma unroll
                for (int pp = 0; pp < NH; ++pp) {
                    const int p = NH * h + pp;
                    const int i0 = 4 * EPL * p + EPL * g;
                    const typename K::ld_t av = *reinterpret_cast<const typename K::ld_t *>(pr + i0);
                    if constexpr (BF) {
                        const u4v xah = *reinterpret_cast<const u4v *>(&L.xi[(a * 16 + n) * TB + i0]);
                        const u4v xal = *reinterpret_cast<const u4v *>(&L.xi[XN + (a * 16 + n) * TB + i0]);
                        tacc[b] = mfma(av, xah, tacc[b]);
                        tacc[b] = mfma(av, xal, tacc[b]);
                        if (a != b) {
                            const u4v xbh = *reinterpret_cast<const u4v *>(&L.xi[(b * 16 + n) * TB + i0]);
                            const u4v xbl = *reinterpret_cast<const u4v *>(&L.xi[XN + (b * 16 + n) * TB + i0]);
                            tacc[a] = mfma(av, xbh, tacc[a]);
                            tacc[a] = mfma(av, xbl, tacc[a]);
                        }
                    } else {
#pragma unroll
                        for (int e = 0; e < EPL; ++e) {
                            const X at = av[e];
                            tacc[b] = mfma(at, L.xi[(a * TB + i0 + e) * 16 + n], tacc[b]);
                            if (a != b) tacc[a] = mfma(at, L.xi[(b * TB + i0 + e) * 16 + n], tacc[a]);
                        }
                    }
                }
            }
        }
        if constexpr (NW == 8) {
            // the two halves, added in a fixed order through LDS (the vectors
            // and planes of this tile are no longer read after the barrier)
            __syncthreads();
            A *hbuf = reinterpret_cast<A *>(&L);   // [row group][6 accumulators][64 lanes]
            if (h == 1) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    hbuf[(rg * 6 + a) * 64 + lane] = dacc[a];
                    hbuf[(rg * 6 + 3 + a) * 64 + lane] = tacc[a];
                }
            }
            __syncthreads();
            if (h == 0) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    dacc[a] = dacc[a] + hbuf[(rg * 6 + a) * 64 + lane];
                    tacc[a] = tacc[a] + hbuf[(rg * 6 + 3 + a) * 64 + lane];
                }
            }
        }
        if (h == 0) {
            // entry e of lane (g, n) is bead 16 rg + orow(g, e), vector n
            P *pd = bpart + ((size_t)J * n3pad + (size_t)I * TS) * 16 + n;
            P *pt = bpart + ((size_t)I * n3pad + (size_t)J * TS) * 16 + n;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int bead = 16 * rg + K::orow(g, e);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    pd[(size_t)(3 * bead + a) * 16] = dacc[a][e];
                    if (offd) pt[(size_t)(3 * bead + a) * 16] = tacc[a][e];
                }
            }
        }
    }
}

// Tile arrays that fit the Infinity Cache (TILE_CACHE_BYTES) are read with
// allocating loads, so that they stay resident from one product to the next.
// The persistent grid: as many workgroups as the device holds at once
// (compute units x resident workgroups of this kernel), found once per
// context and precision.
template <typename T, bool CACHED> static auto block_kernel()
{
    return k_block_tiles<T, CACHED>;
}

template <typename T, bool CACHED> static int block_grid(const Ctx &c)
{
    int &g = c.block_wgs[sizeof(T) == 8 ? 0 : sizeof(T) == 4 ? 1 : 2];
    if (g > 0) return g;
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, block_kernel<T, CACHED>(), 64 * BK<T>::NWAVE, 0) !=
            hipSuccess ||
        cus < 1 || per < 1)
        return 256;   // not cached: asked again next time
    g = cus * per;
    return g;
}

template <typename T>
static void block_tiles_launch(const Ctx &c, const T *tiles, hipStream_t s)
{
    const bool cached = (size_t)c.ntiles * TILE6 * sizeof(T) <= TILE_CACHE_BYTES;
    const int cap = cached ? block_grid<T, true>(c) : block_grid<T, false>(c);
    const int grid = c.ntiles < cap ? c.ntiles : cap;
    const int npad = c.nbt * TB;
    typedef typename BK<T>::x_t X;
    typedef typename BK<T>::part_t P;
    hipEvent_t e0 = c.prof_ev0, e1 = c.prof_ev1;
    c.prof_ev0 = c.prof_ev1 = nullptr;
    if (cached)
        hipExtLaunchKernelGGL((block_kernel<T, true>()), dim3(grid), dim3(64 * BK<T>::NWAVE), 0, s, e0, e1, 0u,
                              c.ntiles, npad, c.n3pad, c.tile_ij, tiles,
                              reinterpret_cast<const X *>(c.xpk), reinterpret_cast<P *>(c.bpart),
                              c.gate);
    else
        hipExtLaunchKernelGGL((block_kernel<T, false>()), dim3(grid), dim3(64 * BK<T>::NWAVE), 0, s, e0, e1, 0u,
                              c.ntiles, npad, c.n3pad, c.tile_ij, tiles,
                              reinterpret_cast<const X *>(c.xpk), reinterpret_cast<P *>(c.bpart),
                              c.gate);
}

void launch_block_tiles(const Ctx &c, int prec, const double *v, int m, hipStream_t s,
                        bool packed)
{
    const int npad = c.nbt * TB;
    const int np = 3 * npad * BLOCK_RHS;
    if (!packed)
        hipLaunchKernelGGL(k_pack_block, dim3((np + 255) / 256), dim3(256), 0, s, c.N, c.n3, npad,
                           m, prec, v, c.xpk, c.vpk, c.gate);
    if (prec == RPY_PREC_BF16) block_tiles_launch<uint16_t>(c, c.p16, s);
    else if (prec == RPY_PREC_F32) block_tiles_launch<float>(c, c.p32, s);
    else block_tiles_launch<double>(c, c.d64, s);
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
// loaded SF_PF quads ahead; six 16x16x4 FP64 MFMAs add
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
// tile partials instead: 16 rows x 16 vectors each, one output per thread
// (rows 16 b .. 16 b + 15, contiguous with the vectors in every slot K).  A
// thread issues the loads of PS_BATCH slots at once, sums them as a pairwise
// tree and adds the batches in K order, in FP64, into ypart[j][row].  This
// HBM stream overlaps the matrix-core work.
constexpr int PS_BATCH = 32;
template <typename P>
__device__ inline void block_part_sum(int b, int n3, int n3pad, int m, int nslot,
                                      const P *__restrict__ part, double *__restrict__ ypart)
{
    const int row = 16 * b + (threadIdx.x >> 4), j = threadIdx.x & 15;
    if (row >= n3 || j >= m) return;
    const P *pp = part + (size_t)row * BLOCK_RHS + j;
    const size_t ks = (size_t)n3pad * BLOCK_RHS;
    double y = 0.0;
    for (int K = 0; K < nslot; K += PS_BATCH) {
        // branch-free: a slot past nslot re-reads the last one and is zeroed
        // after the loads (a conditional load would wait at every join)
        P raw[PS_BATCH];
#pragma unroll
        for (int u = 0; u < PS_BATCH; ++u) raw[u] = pp[(size_t)min(K + u, nslot - 1) * ks];
        double q[PS_BATCH];
#pragma unroll
        for (int u = 0; u < PS_BATCH; ++u) q[u] = K + u < nslot ? (double)raw[u] : 0.0;
#pragma unroll
        for (int h = PS_BATCH / 2; h >= 1; h >>= 1)
#pragma unroll
            for (int u = 0; u < h; ++u) q[u] += q[u + h];
        y += q[0];
    }
    ypart[(size_t)j * n3 + row] = y;
}

__global__ __launch_bounds__(256) void k_block_sf(int nk, int nk16, int nq, int cq, int nkb,
                                                  int N, int n3, int n3pad, int m, int nslot,
                                                  const double2 *eph, const double *vpk,
                                                  double *sfpart,
                                                  const void *__restrict__ part, int part64,
                                                  double *__restrict__ ypart,
                                                  const int *__restrict__ gate)
{
    __shared__ d4v red[SF_WAVES - 1][6][64];
    if (gate && *gate) return;
    if ((int)blockIdx.x >= nkb) {
        const int b = (blockIdx.x - nkb) + blockIdx.y * (gridDim.x - nkb);
        if (part64)
            block_part_sum(b, n3, n3pad, m, nslot, reinterpret_cast<const double *>(part), ypart);
        else
            block_part_sum(b, n3, n3pad, m, nslot, reinterpret_cast<const float *>(part), ypart);
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
    // A ring of SF_PF + 1 buffers in fixed registers: each is loaded SF_PF
    // steps before it is consumed.  A step past the chunk consumes a zero
    // phase.
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
    // Blocks of SF_U steps, each fully unrolled: the prefetches stay inside
    // a block, so no load is in flight across a loop back edge (the
    // compiler then waits for all of them at the loop head) and every wait
    // leaves the next SF_PF steps' loads outstanding.
    const int qa = q0 + w;
    const int nsteps = q1 > qa ? (q1 - qa + S - 1) / S : 0;
    for (int t0 = 0; t0 < nsteps; t0 += SF_U) {
        const int qb = qa + t0 * S;
        SfLd b[SF_PF + 1];
#pragma unroll
        for (int t = 0; t < SF_PF; ++t) fetch(qb + t * S, b[t]);
#pragma unroll
        for (int t = 0; t < SF_U; ++t) {
            // compiler-only barrier: keeps each prefetch where it is written
            // (the loaded values are otherwise forwarded and the loads
            // re-issued where they are consumed)
            if (t + SF_PF < SF_U) fetch(qb + (t + SF_PF) * S, b[(t + SF_PF) % (SF_PF + 1)]);
            __asm__ volatile("" ::: "memory");
            use(b[t % (SF_PF + 1)], qb + t * S);
        }
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

void launch_block_sf(const Ctx &c, int m, int prec, hipStream_t s)
{
    const int nq = (c.N + 3) / 4;
    const int cq = (nq + c.nchb - 1) / c.nchb;
    const int nkb = (c.nk + 15) / 16;
    // grid x: nkb structure-factor blocks, then ceil(npg / nchb) part-sum
    // workgroups per grid row (npg = groups of 16 rows)
    const int npg = (c.n3 + 15) / 16;
    const int px = (npg + c.nchb - 1) / c.nchb;
    hipLaunchKernelGGL(k_block_sf, dim3(nkb + px, c.nchb), dim3(64 * SF_WAVES), 0, s, c.nk,
                       (c.nk + 15) / 16 * 16, nq, cq, nkb, c.N, c.n3, c.n3pad, m, c.nbt, c.eph,
                       c.vpk, c.sfpart, (const void *)c.bpart, prec == RPY_PREC_F64 ? 1 : 0,
                       c.ypart, c.gate);
    const int nt = (c.nk + 15) / 16 * 2 * BLOCK_RHS * 16;
    hipLaunchKernelGGL(k_block_sf_reduce, dim3((nt + 255) / 256), dim3(256), 0, s, c.nk, c.nchb,
                       c.kcoef, c.sfpart, c.tkm, c.gate);
}

// ------------------------------ back-projection + partial sum + epilogue
// Workgroup: 16 beads nu0 .. nu0 + 15, EPI_W waves; wave w takes the
// wave-vector steps w, w + EPI_W, ... (4 wave vectors each).  Lane (g, i)
// holds the phase of bead nu0 + i and k = 4 step + g (A operand: row =
// bead, inner = k) and T[k][3 half + c][j = i] (B operand; tkm rows >= nk are
// zero), loaded EPI_PF steps ahead; six FP64 MFMAs per step add
//   sum_k cos(k.r) Tc + sin(k.r) Ts,  c = 0..2.
// The waves are summed in a fixed order in LDS; thread (j, bead) adds the
// summed tile partials ypart and applies the epilogue of f.mode (as in
// k_kspace_epi); with f.pack it also writes V_p in the packed layouts, so the
// next product of the series needs no packing launch.
constexpr int EPI_W = 8;
struct EpiLd {
    double2 e;
    double t[6];
};
__global__ __launch_bounds__(64 * EPI_W) void k_block_epi(int N, int n3, int nk4, int nk16,
                                                          const double2 *eph, const double *tkm,
                                                          const double *__restrict__ ypart,
                                                          EpiArgs f, int npad,
                                                          void *__restrict__ xs,
                                                          double *__restrict__ vpk,
                                                          const int *__restrict__ gate)
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
        // the three cos products, then the three sin products: no MFMA waits
        // on the one just issued
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
            acc[cc] = __builtin_amdgcn_mfma_f64_16x16x4f64(c, d.t[cc], acc[cc], 0, 0, 0);
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
            acc[cc] = __builtin_amdgcn_mfma_f64_16x16x4f64(sn, d.t[3 + cc], acc[cc], 0, 0, 0);
    };
    constexpr int S = EPI_W;
    // blocks of EPI_U fully unrolled steps, as in k_block_sf
    const int nsteps = (nst - w + S - 1) / S;
    for (int t0 = 0; t0 < nsteps; t0 += EPI_U) {
        const int sb = w + t0 * S;
        EpiLd b[EPI_PF + 1];
#pragma unroll
        for (int t = 0; t < EPI_PF; ++t) fetch(sb + t * S, b[t]);
#pragma unroll
        for (int t = 0; t < EPI_U; ++t) {
            if (t + EPI_PF < EPI_U) fetch(sb + (t + EPI_PF) * S, b[(t + EPI_PF) % (EPI_PF + 1)]);
            __asm__ volatile("" ::: "memory");
            use(b[t % (EPI_PF + 1)], sb + t * S);
        }
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
            if (f.pack) pack_entry(f.pack_prec, npad, bead, c, j, v1, xs, vpk);
        } else {
            const double vp = 2.0 * (ya * yy - yb * f.vprev[o]) - f.vprev2[o];
            f.vout[o] = vp;
            f.acc[o] += f.scal[8 + f.p] * vp;
            if (f.pack) pack_entry(f.pack_prec, npad, bead, c, j, vp, xs, vpk);
        }
    }
}

void launch_block_epi(const Ctx &c, const EpiArgs &f, hipStream_t s)
{
    hipLaunchKernelGGL(k_block_epi, dim3((c.N + 15) / 16), dim3(64 * EPI_W), 0, s, c.N, c.n3,
                       c.nk4, (c.nk + 15) / 16 * 16, c.eph, c.tkm, c.ypart, f, c.nbt * TB, c.xpk,
                       c.vpk, c.gate);
}

}  // namespace rpy
