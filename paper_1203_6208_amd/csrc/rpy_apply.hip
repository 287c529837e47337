// rpy_apply.hip -- the product y = D.V (stored real-space tiles + reciprocal
// sum per product) and the Fixman-Chebyshev recurrence epilogue
// (arXiv:1203.6208, eq. DFmodified and eq. cheb1-cheb3).
#include <hip/hip_ext.h>

#include "rpy_internal.h"
#include "rpy_sf.h"

namespace rpy {

#define RPY_RHS_GROUPS(m, BODY)                                              \
    for (int j0 = 0; j0 < (m);) {                                            \
        const int mc = ((m) - j0) >= 4 ? 4 : ((m) - j0);                     \
        if (mc == 4) { constexpr int MC = 4; BODY; }                         \
        else if (mc == 3) { constexpr int MC = 3; BODY; }                    \
        else if (mc == 2) { constexpr int MC = 2; BODY; }                    \
        else { constexpr int MC = 1; BODY; }                                 \
        j0 += mc;                                                            \
    }

// ------------------------------------------------------------------ SYMV
template <typename A> __device__ inline A sum16(A x)
{
#pragma unroll
    for (int o = 8; o >= 1; o >>= 1) x += __shfl_xor(x, o, 16);
    return x;
}

// Loads of a packed plane row (64 values of one bead row and one entry of
// the 3 x 3 blocks): lane q (0..15) of a 16-lane row group owns the bead
// columns col(q, e), e = 0..3, read with 16-byte (FP64, FP32) or 8-byte
// (BF16) loads that are contiguous across the row group: allocating loads
// when CACHED, else non-temporal ones.
template <typename T> struct P6;
template <> struct P6<double> {
    typedef double d2v __attribute__((ext_vector_type(2)));
    struct raw_t {
        d2v u, v;
    };
    static constexpr bool hoist = false;
    __device__ static int col(int q, int e) { return 32 * (e >> 1) + 2 * q + (e & 1); }
    template <bool CACHED> __device__ static raw_t raw(const double *row, int q)
    {
        const d2v *a = reinterpret_cast<const d2v *>(row + 2 * q);
        const d2v *b = reinterpret_cast<const d2v *>(row + 32 + 2 * q);
        if constexpr (CACHED) return {*a, *b};
        else return {__builtin_nontemporal_load(a), __builtin_nontemporal_load(b)};
    }
    __device__ static void cvt(const raw_t &r, double a[4])
    {
        a[0] = r.u.x;
        a[1] = r.u.y;
        a[2] = r.v.x;
        a[3] = r.v.y;
    }
};
template <> struct P6<float> {
    typedef float raw_t __attribute__((ext_vector_type(4)));
    static constexpr bool hoist = false;
    __device__ static int col(int q, int e) { return 4 * q + e; }
    template <bool CACHED> __device__ static raw_t raw(const float *row, int q)
    {
        const raw_t *a = reinterpret_cast<const raw_t *>(row + 4 * q);
        if constexpr (CACHED) return *a;
        else return __builtin_nontemporal_load(a);
    }
    __device__ static void cvt(const raw_t &u, double a[4])
    {
        a[0] = u.x;
        a[1] = u.y;
        a[2] = u.z;
        a[3] = u.w;
    }
};
template <> struct P6<uint16_t> {
    typedef uint32_t raw_t __attribute__((ext_vector_type(2)));
    static constexpr bool hoist = true;
    __device__ static int col(int q, int e) { return 4 * q + e; }
    template <bool CACHED> __device__ static raw_t raw(const uint16_t *row, int q)
    {
        const raw_t *a = reinterpret_cast<const raw_t *>(row + 4 * q);
        if constexpr (CACHED) return *a;
        else return __builtin_nontemporal_load(a);
    }
    __device__ static void cvt(const raw_t &u, double a[4])
    {
        a[0] = __uint_as_float(u.x << 16);
        a[1] = __uint_as_float(u.x & 0xFFFF0000u);
        a[2] = __uint_as_float(u.y << 16);
        a[3] = __uint_as_float(u.y & 0xFFFF0000u);
    }
};

// Product on the packed tiles (6 planes per bead row, tile[t][i][c][j]),
// FP64, FP32 or BF16 entries, FP64 arithmetic.  nsf workgroups (at the
// front of the launch or spread through it) compute T_k of v for a few wave
// vectors each (sf_direct_block); each further workgroup (NW waves) takes
// one stored tile (I, J), in stored order or, when `flip`, in reverse order
// (each tile's results go to its own slots, so the order changes no value).
// Wave w, row group g (16 lanes), lane q: bead rows i = 4 NW it + 4 w + g
// (it < 16 / NW); lane q owns the bead columns jb(e) = P6<T>::col(q, e),
// e = 0..3, of every plane.  With B the symmetric 3 x 3 block of (i, j), the
// row sums of B x_j over the 16 lanes give A_IJ x_J -> part[J][j][rows of I];
// for off-diagonal tiles each lane also accumulates B x_i for its columns,
// and the 4 row groups and the NW waves are combined in a fixed order ->
// part[I][j][rows of J].  Diagonal tiles hold both (i, j) and (j, i) and
// take row sums only.
// Four vectors need 274 VGPRs, one wave per SIMD; capped at 256 (two waves,
// a few spills) the FP64 launch takes 132 us instead of 176 us at N = 4000.
// Three and four vectors run at two waves per SIMD.
// Waves per tile workgroup: 4, or 2 for BF16 tiles with one vector.  Those
// short, cache-resident rows are latency-bound: two waves of 32 rows each,
// every next row loaded while the current one is used, take 28.5 us at
// N = 4000 against 32.3 us for four waves with all of a lane's rows loaded
// at once (one wave: 41.6 us, eight: 38.6 us).  FP32 tiles keep four waves
// (37.6 us; two: 38.1 us).
template <typename T, int M> constexpr int symv_waves() { return sizeof(T) == 2 && M == 1 ? 2 : 4; }

template <typename T, int M, bool CACHED, int NW = symv_waves<T, M>()>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(M >= 3 ? 2 : 1, 8))) void k_symv6(int N, int n3, int n3pad, int rhs_cap, int j0,
                                               int nsf, int sfr, int flip, int nk,
                                               double invL,
                                               const KVec *__restrict__ kvec,
                                               const KCoef *__restrict__ kcoef,
                                               const double *__restrict__ rt,
                                               double *__restrict__ tk,
                                               const int2 *__restrict__ tile_ij,
                                               const T *__restrict__ tiles,
                                               const double *__restrict__ v,
                                               double *__restrict__ part,
                                               const int *__restrict__ gate)
{
    extern __shared__ double smem[];
    if (gate && *gate) return;   // a product past the settled adaptive order
    // workgroup b is structure-factor workgroup b / sfr when b is a multiple
    // of sfr below nsf sfr, else tile ordinal b - (structure-factor
    // workgroups up to b): sfr = 1 puts them at the front of the launch,
    // larger sfr spreads them through it
    const int bid = blockIdx.x, ntl = (int)gridDim.x - nsf;
    if (bid % sfr == 0 && bid / sfr < nsf) {
        sf_direct_block<M, NW>(bid / sfr, N, nk, rhs_cap, j0, invL, n3, kvec, kcoef, rt, v, tk, smem);
        return;
    }
    double(*sx)[TS] = reinterpret_cast<double(*)[TS]>(smem);                    // [M][TS]
    double(*scol)[M][TS] = reinterpret_cast<double(*)[M][TS]>(smem + M * TS);  // [NW][M][TS]
    constexpr int NT = 64 * NW, RPI = 4 * NW, NIT = TB / RPI;   // threads, rows per pass, passes
    constexpr bool HOIST = P6<T>::hoist && NW == 4;
    const int ord = bid - min(nsf, bid / sfr + 1);
    const int t = flip ? ntl - 1 - ord : ord;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane >> 4, q = lane & 15;
    // BF16 rows of several vectors are small: all four of a lane's rows
    // are loaded before any arithmetic (more bytes in flight per wave;
    // 34.1 against 37.4 us at N = 4000 for one vector, before it moved to two
    // waves).  FP64 rows of one-vector products, and the BF16 rows of the
    // two-wave form, are loaded one row ahead, each while the previous one
    // is used (FP64: 67.2 against 69.2 us at N = 4000, at two waves per SIMD
    // instead of three); FP32 rows and the rows of several vectors one at a
    // time (hoisting them costs occupancy: FP32 46.9 against 43.8 us).  The
    // tile's address needs only t, so the first row is loaded before the
    // vector loads, which wait on the tile's (I, J) (FP32 one-vector steps
    // 577 -> 582 per second; all four hoisted BF16 rows issued there lose:
    // 32.2 -> 33.1 us).
    const T *tile = tiles + (size_t)t * TILE6;
    typename P6<T>::raw_t rw[NIT][6];
    constexpr bool PF = !HOIST && M == 1 && (sizeof(T) == 8 || NW < 4);   // rows one ahead
    if constexpr (!HOIST) {
#pragma unroll
        for (int c = 0; c < 6; ++c)
            rw[0][c] = P6<T>::template raw<CACHED>(tile + (size_t)(4 * w + g) * 6 * TB + c * TB, q);
    }
    const int2 ij = tile_ij[t];
    const int I = ij.x, J = ij.y;
    // the vector loads of x_I (for LDS) and x_J (registers) all go out
    // before the first LDS store, which waits for them
    constexpr int NSX = (M * TS + NT - 1) / NT;
    double sxv[NSX];
#pragma unroll
    for (int u = 0; u < NSX; ++u) {
        const int e = threadIdx.x + NT * u, j = e / TS, row = I * TS + e % TS;
        sxv[u] = e < M * TS && row < n3 ? v[(size_t)(j0 + j) * n3 + row] : 0.0;
    }
    double xj[M][4][3];
#pragma unroll
    for (int j = 0; j < M; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int col = J * TS + 3 * P6<T>::col(q, e) + c;
                xj[j][e][c] = col < n3 ? v[(size_t)(j0 + j) * n3 + col] : 0.0;
            }
#pragma unroll
    for (int u = 0; u < NSX; ++u) {
        const int e = threadIdx.x + NT * u;
        if (e < M * TS) sx[e / TS][e % TS] = sxv[u];
    }
    double cacc[M][4][3];
#pragma unroll
    for (int j = 0; j < M; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) cacc[j][e][0] = cacc[j][e][1] = cacc[j][e][2] = 0.0;
    __syncthreads();
    const bool offd = I != J;
    if constexpr (HOIST) {
#pragma unroll
        for (int it = 0; it < NIT; ++it)
#pragma unroll
            for (int c = 0; c < 6; ++c)
                rw[it][c] = P6<T>::template raw<CACHED>(
                    tile + (size_t)(RPI * it + 4 * w + g) * 6 * TB + c * TB, q);
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int i = RPI * it + 4 * w + g;
        double b[6][4];
        if constexpr (PF) {
            if (it + 1 < NIT) {
#pragma unroll
                for (int c = 0; c < 6; ++c)
                    rw[it + 1][c] = P6<T>::template raw<CACHED>(
                        tile + (size_t)(i + RPI) * 6 * TB + c * TB, q);
            }
            // compiler-only barrier: keeps the next row's loads ahead of this
            // row's arithmetic
            __asm__ volatile("" ::: "memory");
        } else if constexpr (!HOIST) {
            if (it > 0) {
#pragma unroll
                for (int c = 0; c < 6; ++c)
                    rw[it][c] = P6<T>::template raw<CACHED>(tile + (size_t)i * 6 * TB + c * TB, q);
            }
        }
#pragma unroll
        for (int c = 0; c < 6; ++c) P6<T>::cvt(rw[it][c], b[c]);
#pragma unroll
        for (int j = 0; j < M; ++j) {
            double r0 = 0.0, r1 = 0.0, r2 = 0.0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double x0 = xj[j][e][0], x1 = xj[j][e][1], x2 = xj[j][e][2];
                r0 += b[0][e] * x0 + b[1][e] * x1 + b[2][e] * x2;
                r1 += b[1][e] * x0 + b[3][e] * x1 + b[4][e] * x2;
                r2 += b[2][e] * x0 + b[4][e] * x1 + b[5][e] * x2;
            }
            r0 = sum16(r0);
            r1 = sum16(r1);
            r2 = sum16(r2);
            if (q < 3)
                part[((size_t)J * rhs_cap + j0 + j) * n3pad + I * TS + 3 * i + q] =
                    q == 0 ? r0 : q == 1 ? r1 : r2;
            if (offd) {
                const double y0 = sx[j][3 * i], y1 = sx[j][3 * i + 1], y2 = sx[j][3 * i + 2];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    cacc[j][e][0] += b[0][e] * y0 + b[1][e] * y1 + b[2][e] * y2;
                    cacc[j][e][1] += b[1][e] * y0 + b[3][e] * y1 + b[4][e] * y2;
                    cacc[j][e][2] += b[2][e] * y0 + b[4][e] * y1 + b[5][e] * y2;
                }
            }
        }
    }
    if (!offd) return;
    // combine the 4 row groups of a wave, then the 4 waves through LDS
#pragma unroll
    for (int j = 0; j < M; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double s = cacc[j][e][c];
                s += __shfl_xor(s, 16);
                s += __shfl_xor(s, 32);
                if (g == 0) scol[w][j][3 * P6<T>::col(q, e) + c] = s;
            }
    __syncthreads();
    for (int e = threadIdx.x; e < M * TS; e += blockDim.x) {
        const int j = e / TS, cidx = e % TS;
        double s = scol[0][j][cidx];
#pragma unroll
        for (int w2 = 1; w2 < NW; ++w2) s += scol[w2][j][cidx];
        part[((size_t)I * rhs_cap + j0 + j) * n3pad + J * TS + cidx] = s;
    }
}

template <typename T, int M> static size_t symv_lds(const Ctx &)
{
    // sx occupies M*TS double slots (whatever A is), then scol[NW][M][TS];
    // the structure-factor workgroups use NW x 6 KPW M doubles
    constexpr int NW = symv_waves<T, M>();
    const size_t tile = sizeof(double) * M * TS + sizeof(double) * NW * M * TS;
    const size_t sf = sizeof(double) * NW * 6 * sf_kpw<M>() * M;
    return tile > sf ? tile : sf;
}

template <typename T, int M>
static void symv_launch(const Ctx &c, const T *tiles, const double *v, int j0, hipStream_t s)
{
    const int nsf = (c.nk + sf_kpw<M>() - 1) / sf_kpw<M>();
    // The structure-factor workgroups' sincospi work: spread through the FP64
    // tile stream it overlaps best (68.7 against 70.0 us at the front, N =
    // 4000); the shorter, cache-resident FP32 / BF16 streams do better with
    // it at the front (BF16 32.2 against 35.1 us spread)
    const int sfr = sizeof(T) == 8 ? (nsf + c.ntiles) / nsf : 1;
    const size_t lds = symv_lds<T, M>(c);
    // Allocating loads, with the tile order reversed on every other launch,
    // for arrays that fit the Infinity Cache (each product then starts on the
    // tiles the previous one read last); otherwise non-temporal loads in
    // stored order, which keep the stream from evicting the rest.
    const size_t bytes = (size_t)c.ntiles * TILE6 * sizeof(T);
    const bool cached = bytes <= TILE_CACHE_BYTES;
    const int flip = cached ? (int)(c.symv_calls++ & 1u) : 0;
    // when profiled, the dispatch itself records the start and end events,
    // so that they time the kernel alone (null events: a plain launch)
    hipEvent_t e0 = c.prof_ev0, e1 = c.prof_ev1;
    c.prof_ev0 = c.prof_ev1 = nullptr;
    if (cached)
        hipExtLaunchKernelGGL((k_symv6<T, M, true>), dim3(nsf + c.ntiles), dim3(64 * symv_waves<T, M>()),
                              (uint32_t)lds, s, e0, e1, 0u, c.N, c.n3, c.n3pad, c.rhs_cap, j0, nsf,
                              sfr, flip, c.nk, c.pc.invL, c.kvec, c.kcoef, c.rt, c.tk, c.tile_ij,
                              tiles, v, c.part, c.gate);
    else
        hipExtLaunchKernelGGL((k_symv6<T, M, false>), dim3(nsf + c.ntiles), dim3(64 * symv_waves<T, M>()),
                              (uint32_t)lds, s, e0, e1, 0u, c.N, c.n3, c.n3pad, c.rhs_cap, j0, nsf,
                              sfr, flip, c.nk, c.pc.invL, c.kvec, c.kcoef, c.rt, c.tk, c.tile_ij,
                              tiles, v, c.part, c.gate);
}

template <typename T>
static void symv_group(const Ctx &c, const T *tiles, const double *v, int j0, int mc,
                       hipStream_t s)
{
    if (mc == 4) symv_launch<T, 4>(c, tiles, v, j0, s);
    else if (mc == 3) symv_launch<T, 3>(c, tiles, v, j0, s);
    else if (mc == 2) symv_launch<T, 2>(c, tiles, v, j0, s);
    else symv_launch<T, 1>(c, tiles, v, j0, s);
}

void launch_symv(const Ctx &c, int prec, const double *v, int j0, int mc, hipStream_t s)
{
    if (prec == RPY_PREC_F32)
        symv_group<float>(c, c.p32, v, j0, mc, s);
    else if (prec == RPY_PREC_BF16)
        symv_group<uint16_t>(c, c.p16, v, j0, mc, s);
    else
        symv_group<double>(c, c.d64, v, j0, mc, s);
}

// ------------------------------------------------- structure-factor reduction
// Workgroup (16 wave vectors) x (64 chunk groups: 16 waves x 4 lane quarters);
// grid (k blocks, 2 M): y = (rhs j, cos or sin half).  Lane quarter `sub` of
// wave g sums the chunks 4 g + sub, +64, ...; an xor tree over the quarters
// and the 16 waves in LDS combine them in a fixed order, then
//   T_k = 2 m(k) (I - khat khat) C_k  (or S_k)
// goes to tk[k][j][3 half + c].
__global__ __launch_bounds__(1024) void k_sf_reduce(int nk, int nsfc, int rhs_cap, int j0,
                                                    const KCoef *__restrict__ kcoef,
                                                    const double *__restrict__ sfpart,
                                                    double *__restrict__ tk,
                                                    const int *__restrict__ gate)
{
    __shared__ double red[16][3][16];
    if (gate && *gate) return;
    const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int kk = lane & 15, sub = lane >> 4;
    const int k = blockIdx.x * 16 + kk;
    const int j = blockIdx.y >> 1, half = blockIdx.y & 1;
    // the projection of the 16 threads that finish, loaded with the
    // partials (after the barrier it would be a second memory round trip)
    KCoef kc = {0.0, 0.0, 0.0, 0.0};
    if (threadIdx.x < 16 && k < nk) kc = kcoef[k];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (k < nk) {
        const size_t cstride = (size_t)6 * rhs_cap * nk;
        const double *o = sfpart + (size_t)(6 * (j0 + j) + 3 * half) * nk + k;
        for (int ch = 4 * g + sub; ch < nsfc; ch += 64) {
            s0 += o[ch * cstride];
            s1 += o[ch * cstride + nk];
            s2 += o[ch * cstride + 2 * (size_t)nk];
        }
    }
    s0 += __shfl_xor(s0, 16);
    s0 += __shfl_xor(s0, 32);
    s1 += __shfl_xor(s1, 16);
    s1 += __shfl_xor(s1, 32);
    s2 += __shfl_xor(s2, 16);
    s2 += __shfl_xor(s2, 32);
    if (sub == 0) {
        red[g][0][kk] = s0;
        red[g][1][kk] = s1;
        red[g][2][kk] = s2;
    }
    __syncthreads();
    if (threadIdx.x >= 16 || k >= nk) return;
    double t[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double a = 0.0;
#pragma unroll
        for (int w = 0; w < 16; ++w) a += red[w][c][kk];
        t[c] = a;
    }
    const double h = kc.hx * t[0] + kc.hy * t[1] + kc.hz * t[2];
    double *o = tk + ((size_t)k * rhs_cap + j0 + j) * 6 + 3 * half;
    o[0] = kc.w * (t[0] - kc.hx * h);
    o[1] = kc.w * (t[1] - kc.hy * h);
    o[2] = kc.w * (t[2] - kc.hz * h);
}

void launch_sf_reduce(const Ctx &c, int m, hipStream_t s)
{
    RPY_RHS_GROUPS(m, hipLaunchKernelGGL(k_sf_reduce, dim3((c.nk + 15) / 16, 2 * MC), dim3(1024),
                                         0, s, c.nk, c.nsfc, c.rhs_cap, j0, c.kcoef, c.sfpart,
                                         c.tk, c.gate));
}

// ------------------------------------- reciprocal back-projection + epilogue
// Workgroup: 16 beads x 64 slices (16 waves; lane = bead (low 4 bits) and
// sub-slice (high 2 bits); slice u = 4 wave + sub).  Slice u owns the wave
// vectors [u nk/64, (u+1) nk/64) and the tile columns K = u, u+64, ...:
//   y_u = sum_K part[K][j][3 nu + c] + sum_k cos(k.r_nu) Tc_k + sin(k.r_nu) Ts_k
// with k.r_nu = 2 pi n.s_nu.  The wave vectors are sorted by (n_x, n_y) and
// then n_z, so inside a run of equal (n_x, n_y) the phase advances by
// e^{i 2 pi s_z}; a run starts from the product of the bead's phase-table
// entries (staged in LDS), with no transcendental call.  Slices are combined in a fixed order (xor tree over the
// sub-slices, then the 16 waves in LDS), then the epilogue of `mode`:
//   EPI_APPLY      out = y
//   EPI_CHEB_FIRST V_1 = ya y - yb V_0, acc = (c_0/2) V_0 + c_1 V_1, dv = y
//   EPI_CHEB_NEXT  V_p = 2 (ya y - yb V_{p-1}) - V_{p-2}, acc += c_p V_p
//   EPI_ADJ        adjoint step mu_p = c_p g + 2 (ya y - yb mu_{p+1}) - mu_{p+2}
//                  (g = acc, read only; mu_{p+2} = 0 when vprev2 is null),
//                  dv = xs ya mu_p
constexpr int EPI_BEADS = 16;
constexpr int EPI_SLICES = 64;
// When `staged` (nk <= 1024, at most epi_stage_per<M>() x 1024 values of tk,
// and the tables fit the workgroup's LDS), the wave vectors and this
// launch's 6 M values of tk per k are copied to LDS once per workgroup --
// [nk + 1] KVec then [nk][M][6] + 1 -- with every load issued before the
// first LDS write (clamped indices; the copies of the clamped loads land in
// the slack entries, so no write is conditional).  The per-thread counts
// cover the 618 half-space wave vectors of alpha L = 6 for 1-4 vectors.
template <int M> constexpr int epi_stage_per() { return M == 1 ? 6 : M == 2 ? 8 : M == 3 ? 11 : 15; }
constexpr size_t EPI_RED_BYTES = sizeof(double) * 16 * 3 * EPI_BEADS;   // static `red`
template <int M>
__global__ __launch_bounds__(1024) void k_kspace_epi(int N, int n3, int n3pad, int nbt, int nk,
                                                     int nmax, int rhs_cap, int j0, int staged,
                                                     const KVec *kvec,
                                                     const double2 *__restrict__ etab,
                                                     const double *__restrict__ part,
                                                     const double *tk_g, EpiArgs f,
                                                     const int *__restrict__ gate)
{
    __shared__ double red[16][3][EPI_BEADS];
    extern __shared__ double lds[];
    if (gate && *gate) return;
    const int nm1 = nmax + 1;
    double2 *tabs = reinterpret_cast<double2 *>(lds);          // [EPI_BEADS][3 nm1]
    double *stage = lds + 2 * EPI_BEADS * 3 * nm1;
    // Loads that do not depend on the staged tables are issued first: the
    // bead's tile-column partials and, for the 3 EPI_BEADS threads that apply
    // the epilogue, the recurrence operands.
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int bl = lane & 15, sub = lane >> 4;
    const int u = 4 * w + sub;
    const int nu = blockIdx.x * EPI_BEADS + bl;
    const bool live = nu < N;
    double y[M][3];
#pragma unroll
    for (int j = 0; j < M; ++j) y[j][0] = y[j][1] = y[j][2] = 0.0;
    if (live) {
        for (int K = u; K < nbt; K += EPI_SLICES) {
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const double *pp = part + ((size_t)K * rhs_cap + j0 + j) * n3pad + 3 * nu;
                y[j][0] += pp[0];
                y[j][1] += pp[1];
                y[j][2] += pp[2];
            }
        }
    }
    const int eb = (int)threadIdx.x / 3, ec = (int)threadIdx.x % 3;
    const int ebead = blockIdx.x * EPI_BEADS + eb;
    const bool eth = threadIdx.x < 3 * EPI_BEADS && ebead < N;
    double pv[M], pv2[M], pa[M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const size_t o = (size_t)(j0 + j) * n3 + 3 * (size_t)ebead + ec;
        pv[j] = eth && f.mode != EPI_APPLY ? f.vprev[o] : 0.0;
        pv2[j] = eth && f.vprev2 && (f.mode == EPI_CHEB_NEXT || f.mode == EPI_ADJ) ? f.vprev2[o]
                                                                                    : 0.0;
        pa[j] = eth && (f.mode == EPI_CHEB_NEXT || f.mode == EPI_ADJ) ? f.acc[o] : 0.0;
    }
    // the phase tables e^{i 2 pi j s_a} of the workgroup's beads (zero past N)
    const int ntab = EPI_BEADS * 3 * nm1;
    const size_t tab0 = (size_t)blockIdx.x * EPI_BEADS * 3 * nm1;
    const int nlive = min(EPI_BEADS, N - (int)blockIdx.x * EPI_BEADS) * 3 * nm1;
    for (int e = threadIdx.x; e < ntab; e += blockDim.x)
        tabs[e] = e < nlive ? etab[tab0 + e] : make_double2(0.0, 0.0);
    if (staged) {
        KVec *kd = reinterpret_cast<KVec *>(stage);
        double *td = stage + 2 * (nk + 1);
        const int ntk = nk * 6 * M;
        const KVec kv0 = kvec[min((int)threadIdx.x, nk - 1)];
        constexpr int SP = epi_stage_per<M>();
        double tv[SP];
#pragma unroll
        for (int i = 0; i < SP; ++i) {
            const int e = min((int)threadIdx.x + 1024 * i, ntk - 1);
            const int k = e / (6 * M), r = e % (6 * M);
            tv[i] = tk_g[((size_t)k * rhs_cap + j0) * 6 + r];
        }
        kd[min((int)threadIdx.x, nk)] = kv0;
#pragma unroll
        for (int i = 0; i < SP; ++i) td[min((int)threadIdx.x + 1024 * i, ntk)] = tv[i];
    }
    __syncthreads();
    const int klo = (int)((long)u * nk / EPI_SLICES), khi = (int)((long)(u + 1) * nk / EPI_SLICES);
    const double2 *tb = tabs + bl * 3 * nm1;
    const double2 ez = nm1 > 1 ? tb[2 * nm1 + 1] : make_double2(1.0, 0.0);   // e^{i 2 pi s_z}
    const double ezr = ez.x, ezi = ez.y;
    // The loop is written out once per source of the tables, so that each
    // copy reads through a pointer of known address space (LDS reads when
    // staged; a pointer that may be either compiles to generic loads).
    auto kloop = [&](const KVec *kv_s, const double *tk_s, int tk_ld) {
        double cs = 1.0, sn = 0.0;
        int px = -(1 << 30), py = 0, pz = 0;
        for (int k = klo; k < khi; ++k) {
            const KVec kv = kv_s[k];
            if (kv.nx == px && kv.ny == py && kv.nz == pz + 1) {
                const double c2 = cs * ezr - sn * ezi;
                sn = cs * ezi + sn * ezr;
                cs = c2;
            } else {   // a run start: the phase from the bead's tables
                const double2 e = kphase(kv, tb, nm1);
                cs = e.x;
                sn = e.y;
            }
            px = kv.nx;
            py = kv.ny;
            pz = kv.nz;
            const double *tt = tk_s + (size_t)k * tk_ld;
#pragma unroll
            for (int j = 0; j < M; ++j)
#pragma unroll
                for (int c = 0; c < 3; ++c) y[j][c] += cs * tt[6 * j + c] + sn * tt[6 * j + 3 + c];
        }
    };
    if (staged)
        kloop(reinterpret_cast<const KVec *>(stage), stage + 2 * (nk + 1), 6 * M);
    else
        kloop(kvec, tk_g + (size_t)j0 * 6, 6 * rhs_cap);
    const double ya = f.scal ? f.scal[2] : 0.0, yb = f.scal ? f.scal[3] : 0.0;
    // the fused trial, as k_trial_sum: skipped once the order is settled or
    // below the call's first order
    const bool trial = f.trial_n > 0 && (f.mode == EPI_CHEB_FIRST || f.mode == EPI_CHEB_NEXT) &&
                       !f.adapt->done && f.trial_n >= f.adapt->n_start;
#pragma unroll
    for (int j = 0; j < M; ++j) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double v = y[j][c];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if (sub == 0) red[w][c][bl] = v;
        }
        __syncthreads();
        double ta = 0.0, tb2 = 0.0;   // this entry's share of the trial's dot products
        if (eth) {
            double yy = 0.0;
#pragma unroll
            for (int ww = 0; ww < 16; ++ww) yy += red[ww][ec][eb];
            const size_t o = (size_t)(j0 + j) * n3 + 3 * (size_t)ebead + ec;
            double vnew = 0.0;   // the vector this epilogue produces
            if (f.mode == EPI_APPLY) {
                f.vout[o] = yy;
            } else if (f.mode == EPI_CHEB_FIRST) {
                const double v0 = pv[j];
                const double v1 = ya * yy - yb * v0;
                f.vout[o] = v1;
                f.acc[o] = 0.5 * f.scal[8] * v0 + f.scal[9] * v1;
                if (f.dv) f.dv[o] = yy;
                vnew = v1;
            } else if (f.mode == EPI_CHEB_NEXT) {
                const double vp = 2.0 * (ya * yy - yb * pv[j]) - pv2[j];
                f.vout[o] = vp;
                f.acc[o] = pa[j] + f.scal[8 + f.p] * vp;
                vnew = vp;
            } else {
                const double mp = f.scal[8 + f.p] * pa[j] + 2.0 * (ya * yy - yb * pv[j]) - pv2[j];
                f.vout[o] = mp;
                f.dv[o] = f.xs * ya * mp;
            }
            if (trial) {   // the terms in k_trial_sum's order; V_p from the register
                const double *vh = f.vhist + o;
                const double v0 = vh[0];
                double d = -0.5 * f.scal[8] * v0;
                // eight stored terms loaded at a time (a load per term
                // in turn left each trial's epilogue at about 18 us)
                for (int q0 = 0; q0 < f.trial_n; q0 += 8) {
                    double t[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int q = q0 + u;
                        t[u] = q < f.trial_n && q != f.p ? vh[(size_t)q * f.ps] : vnew;
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        if (q0 + u < f.trial_n) d += f.scal[8 + q0 + u] * t[u];
                }
                f.ds[o] = d;
                ta = d * d;
                tb2 = v0 * f.ddw[o];
            }
        }
        if (trial && w == 0) {   // the 3 EPI_BEADS entries are lanes of the first wave
#pragma unroll
            for (int o2 = 32; o2 >= 1; o2 >>= 1) {
                ta += __shfl_xor(ta, o2);
                tb2 += __shfl_xor(tb2, o2);
            }
            if (lane == 0) {
                double *tp = f.tpart + ((size_t)(j0 + j) * gridDim.x + blockIdx.x) * 2;
                tp[0] = ta;
                tp[1] = tb2;
            }
        }
        if (j + 1 < M) __syncthreads();   // red is rewritten by the next vector
    }
}

void launch_kspace_epi(const Ctx &c, const EpiArgs &f, hipStream_t s)
{
    const dim3 g((c.N + EPI_BEADS - 1) / EPI_BEADS), b(1024);
    const size_t tabs = sizeof(double) * 2 * EPI_BEADS * 3 * (size_t)(c.nmax + 1);
    RPY_RHS_GROUPS(f.m, {
        const size_t lds = sizeof(double) * ((size_t)c.nk * (2 + 6 * MC) + 3);
        const int staged = c.nk <= 1024 &&
                           (size_t)c.nk * 6 * MC <= (size_t)1024 * epi_stage_per<MC>() &&
                           tabs + lds + EPI_RED_BYTES <= (size_t)c.lds_max;
        hipLaunchKernelGGL(k_kspace_epi<MC>, g, b, tabs + (staged ? lds : 0), s, c.N, c.n3,
                           c.n3pad, c.nslot, c.nk, c.nmax, c.rhs_cap, j0, staged, c.kvec, c.etab,
                           c.part, c.tk, f, c.gate);
    });
}

// ------------------------------------------------- Chebyshev coefficients
// scal[0] = d_min, scal[1] = d_max, scal[2] = 2/(d_max - d_min),
// scal[3] = (d_max + d_min)/(d_max - d_min), scal[8 + p] = c_p with
//   c_p = (2/n) sum_{j=1..n} sqrt(h x_j + m) cos(p theta_j),
//   theta_j = pi (j - 1/2)/n, x_j = cos theta_j, h = (d_max-d_min)/2, m = (d_max+d_min)/2.
// One 1024-thread workgroup: wave w sums the nodes of coefficients
// p = w, w+16, ... with a lane-parallel sum in a fixed order.
__device__ void cheb_coeffs_block(int n, double lo, double hi, double *__restrict__ scal)
{
    const double h = 0.5 * (hi - lo), mid = 0.5 * (hi + lo);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int p = w; p < n; p += 16) {
        double s = 0.0;
        for (int j = 1 + lane; j <= n; j += 64) {
            const double u = (j - 0.5) / n;
            s += sqrt(h * cospi(u) + mid) * cospi(p * u);
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
        if (lane == 0) scal[8 + p] = 2.0 * s / n;
    }
}

// The interval and the coefficients.  rule = RPY_BOUNDS_PAPER derives the
// interval from du = D.U+ first, RPY_BOUNDS_DILUTE from du = [D.U+, D.U-]
// (fixed-order tree reductions).  With st
// (an adaptive call) the order is the call's first one, adapt_floor if >= 2
// or else eq. nint, nint(sqrt(d_max/d_min)) + 1 rounded half away from zero,
// clamped to [2, adapt_max]; the call's state is reset.
__global__ __launch_bounds__(1024) void k_cheb_coeffs(int nbeads, int n, int rule, double C,
                                                      double dmin, double dmax,
                                                      const double *__restrict__ du,
                                                      double *__restrict__ scal,
                                                      int adapt_floor, int adapt_max,
                                                      AdaptState *__restrict__ st)
{
    __shared__ double red[1024];
    __shared__ double bounds[2];
    __shared__ int order;
    const int tid = threadIdx.x;
    if (rule == RPY_BOUNDS_PAPER || rule == RPY_BOUNDS_DILUTE) {
        // U.D.U / 3N for U+ (du[0 .. 3N)) and, for the dilute rule, U-
        // (du[3N .. 6N) = D.U-, signs (-1)^i)
        const int n3 = 3 * nbeads;
        double uf[2];
        for (int q = 0; q < (rule == RPY_BOUNDS_DILUTE ? 2 : 1); ++q) {
            const double *d = du + (size_t)q * n3;
            double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
            int i = tid;
            for (; i + 3 * 1024 < n3; i += 4 * 1024) {
                s0 += q && (i & 1) ? -d[i] : d[i];   // 1024 is even: the four share a sign
                s1 += q && (i & 1) ? -d[i + 1024] : d[i + 1024];
                s2 += q && (i & 1) ? -d[i + 2048] : d[i + 2048];
                s3 += q && (i & 1) ? -d[i + 3072] : d[i + 3072];
            }
            for (; i < n3; i += 1024) s0 += q && (i & 1) ? -d[i] : d[i];
            red[tid] = (s0 + s1) + (s2 + s3);
            __syncthreads();
            for (int h = 512; h > 0; h >>= 1) {
                if (tid < h) red[tid] += red[tid + h];
                __syncthreads();
            }
            uf[q] = red[0] / n3;
            __syncthreads();
        }
        if (tid == 0) {
            if (rule == RPY_BOUNDS_PAPER) {   // eq. fmax, fmin
                const double np6 = pow((double)nbeads, 0.6);
                const double lmax = 0.35 * np6 * uf[0];
                bounds[0] = lmax / (C * np6);
                bounds[1] = lmax;
            } else {   // eq. lmax-lmin-dilute with d_max = 2 lmax, d_min = lmin / 2
                bounds[0] = 0.5 * uf[1];
                bounds[1] = 2.0 * uf[0];
            }
        }
    } else if (tid == 0) {
        bounds[0] = dmin;
        bounds[1] = dmax;
    }
    __syncthreads();
    const double lo = bounds[0], hi = bounds[1];
    if (tid == 0) {
        int k = n;
        if (st) {
            const double r = round(sqrt(hi / lo)) + 1.0;   // compared in FP64: no overflow
            k = adapt_floor >= 2 ? adapt_floor : (r < (double)adapt_max ? (int)r : adapt_max);
            k = k < 2 ? 2 : (k > adapt_max ? adapt_max : k);
            st->done = 0;
            st->n_used = 0;
            st->n_start = k;
            st->last_etol = 0;
        }
        order = k;
    }
    __syncthreads();
    cheb_coeffs_block(order, lo, hi, scal);
    if (tid == 0) {
        scal[0] = lo;
        scal[1] = hi;
        scal[2] = 2.0 / (hi - lo);
        scal[3] = (hi + lo) / (hi - lo);
    }
}

void launch_cheb_coeffs(const Ctx &c, int n_cheb, int rule, double C, double dmin, double dmax,
                        const double *du, hipStream_t s, int adapt_floor, int adapt_max)
{
    hipLaunchKernelGGL(k_cheb_coeffs, dim3(1), dim3(1024), 0, s, c.N, n_cheb, rule, C, dmin,
                       dmax, du, c.scal, adapt_floor, adapt_max,
                       adapt_floor >= 0 ? c.adapt : nullptr);
}

// ------------------------------------------------------ adaptive order
// Trial order n of an adaptive call (eq. nint, then the E_f criterion).
// Both kernels return at once when the call's order is settled or n is below
// its first order.  k_trial_sum: grid (chunks of 256 entries, m);
//   dS = sum_{q<n} c_q V_q - (c_0/2) V_0      (eq. cheb1, c_q in scal[8..])
// and the chunk's dS.dS and dW.(D dW) by a fixed-order tree.
__global__ __launch_bounds__(256) void k_trial_sum(int n3, int n, size_t ps,
                                                   const AdaptState *__restrict__ st,
                                                   const double *__restrict__ scal,
                                                   const double *__restrict__ vh,
                                                   const double *__restrict__ ddw,
                                                   double *__restrict__ ds,
                                                   double *__restrict__ part)
{
    __shared__ double ra[256], rb[256];
    if (st->done || n < st->n_start) return;
    const int j = blockIdx.y, i = blockIdx.x * 256 + threadIdx.x;
    double a = 0.0, b = 0.0;
    if (i < n3) {
        const size_t o = (size_t)j * n3 + i;
        const double v0 = vh[o];
        double d = -0.5 * scal[8] * v0;
        for (int q = 0; q < n; ++q) d += scal[8 + q] * vh[(size_t)q * ps + o];
        ds[o] = d;
        a = d * d;
        b = v0 * ddw[o];
    }
    ra[threadIdx.x] = a;
    rb[threadIdx.x] = b;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            ra[threadIdx.x] += ra[threadIdx.x + h];
            rb[threadIdx.x] += rb[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double *o = part + ((size_t)j * gridDim.x + blockIdx.x) * 2;
        o[0] = ra[0];
        o[1] = rb[0];
    }
}

// k_trial_check (one workgroup): the chunks summed in order per right-hand
// side, E_f = sqrt(|dS.dS - dW.D.dW| / dW.D.dW); the order is settled when
// every E_f < tol or n = nmax (e_f written, statistics updated, the ETOL
// count raised when the tolerance was missed), else the coefficients of
// order n + 1 replace those of order n.
__global__ __launch_bounds__(1024) void k_trial_check(int m, int nchunk, int n, int nmax,
                                                      double tol, AdaptState *__restrict__ st,
                                                      const double *__restrict__ part,
                                                      double *__restrict__ scal,
                                                      double *__restrict__ e_f)
{
    __shared__ double ra[1024], rb[1024];
    __shared__ double ef[MAX_RHS];
    __shared__ int settle;
    if (st->done || n < st->n_start) return;
    const int tid = threadIdx.x;
    for (int j = 0; j < m; ++j) {
        double a = 0.0, b = 0.0;
        for (int c = tid; c < nchunk; c += 1024) {
            a += part[((size_t)j * nchunk + c) * 2];
            b += part[((size_t)j * nchunk + c) * 2 + 1];
        }
        ra[tid] = a;
        rb[tid] = b;
        __syncthreads();
        for (int h = 512; h > 0; h >>= 1) {
            if (tid < h) {
                ra[tid] += ra[tid + h];
                rb[tid] += rb[tid + h];
            }
            __syncthreads();
        }
        if (tid == 0) ef[j] = sqrt(fabs(ra[0] - rb[0]) / rb[0]);
        __syncthreads();
    }
    if (tid == 0) {
        double worst = 0.0;
        for (int j = 0; j < m; ++j) worst = ef[j] > worst ? ef[j] : worst;
        const bool ok = worst < tol;
        settle = ok || n >= nmax;
        if (settle) {
            for (int j = 0; j < m; ++j) e_f[j] = ef[j];
            st->done = 1;
            st->n_used = n;
            st->last_etol = ok ? 0 : 1;
            if (!ok) {
                st->etol += 1;
                st->missed += 1;
            }
            st->calls += 1;
            st->sum_orders += n;
            if (n > st->max_order) st->max_order = n;
        }
    }
    __syncthreads();
    if (!settle) cheb_coeffs_block(n + 1, scal[0], scal[1], scal);
}

void launch_trial(const Ctx &c, int m, int n, int nmax, double tol, size_t ps,
                  const double *ddw, double *ds, double *e_f, hipStream_t s)
{
    const int nchunk = (c.n3 + 255) / 256;
    hipLaunchKernelGGL(k_trial_sum, dim3(nchunk, m), dim3(256), 0, s, c.n3, n, ps, c.adapt,
                       c.scal, c.vhist, ddw, ds, c.tpart);
    hipLaunchKernelGGL(k_trial_check, dim3(1), dim3(1024), 0, s, m, nchunk, n, nmax, tol,
                       c.adapt, c.tpart, c.scal, e_f);
}

void launch_trial_check(const Ctx &c, int m, int n, int nmax, double tol, double *e_f,
                        hipStream_t s)
{
    const int nchunk = (c.N + EPI_BEADS - 1) / EPI_BEADS;   // k_kspace_epi workgroups
    hipLaunchKernelGGL(k_trial_check, dim3(1), dim3(1024), 0, s, m, nchunk, n, nmax, tol,
                       c.adapt, c.tpart, c.scal, e_f);
}

int trial_chunks(int N)
{
    const int a = (3 * N + 255) / 256, b = (N + EPI_BEADS - 1) / EPI_BEADS;
    return a > b ? a : b;
}

// E_f = sqrt(|dS.dS - dW.(D dW)| / dW.(D dW)), one workgroup per RHS.
__global__ __launch_bounds__(256) void k_sqrt_error(int n3, const double *__restrict__ dw,
                                                    const double *__restrict__ ddw,
                                                    const double *__restrict__ ds,
                                                    double *__restrict__ e_f)
{
    __shared__ double r1[256], r2[256];
    const int j = blockIdx.x;
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < n3; i += blockDim.x) {
        const size_t o = (size_t)j * n3 + i;
        a += ds[o] * ds[o];
        b += dw[o] * ddw[o];
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
    if (threadIdx.x == 0) e_f[j] = sqrt(fabs(r1[0] - r2[0]) / r2[0]);
}

void launch_sqrt_error(const Ctx &c, int m, const double *dw, const double *ddw,
                       const double *ds, double *e_f, hipStream_t s)
{
    hipLaunchKernelGGL(k_sqrt_error, dim3(m), dim3(256), 0, s, c.n3, dw, ddw, ds, e_f);
}

__global__ void k_fill(double *p, double v, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_copy(double *dst, const double *src, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}
void launch_fill(double *p, double v, size_t n, hipStream_t s)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
}
void launch_copy(double *dst, const double *src, size_t n, hipStream_t s)
{
    if (n == 0) return;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dst, src, n);
}

}  // namespace rpy
