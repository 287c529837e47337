// rpy_apply.hip -- the product y = D.V (stored real-space tiles + reciprocal
// sum per product) and the Fixman-Chebyshev recurrence epilogue
// (arXiv:1203.6208, eq. DFmodified and eq. cheb1-cheb3).
#include "rpy_internal.h"

namespace rpy {

constexpr int SF_CHUNK = 64;   // beads per structure-factor partial
constexpr int FIN_BEADS = 16;  // beads per finalize workgroup (16 slices each)

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

// ------------------------------------------------------- structure factors
// Partial structure factors of V over one chunk of SF_CHUNK beads:
//   C_k = sum_mu cos(k.r_mu) V_mu,  S_k = sum_mu sin(k.r_mu) V_mu.
// Grid (chunk, k-block); one thread per wave vector; the chunk's phase tables
// and vectors are staged in LDS.  Output sfpart[chunk][(j*6 + comp)][k].
template <int M>
__global__ __launch_bounds__(256) void k_structure_factors(
    int N, int n3, int nk, int nmax, const KVec *__restrict__ kvec,
    const double2 *__restrict__ etab, const double *__restrict__ v, int j0, int max_rhs,
    double *__restrict__ sfpart)
{
    extern __shared__ double smem[];
    const int nm1 = nmax + 1;
    double2 *stab = reinterpret_cast<double2 *>(smem);          // [SF_CHUNK][3*nm1]
    double *sv = smem + 2 * SF_CHUNK * 3 * nm1;                  // [SF_CHUNK][M][3]
    const int chunk = blockIdx.x;
    const int b0 = chunk * SF_CHUNK;
    const int nb = min(SF_CHUNK, N - b0);
    for (int e = threadIdx.x; e < nb * 3 * nm1; e += blockDim.x)
        stab[e] = etab[(size_t)b0 * 3 * nm1 + e];
    for (int e = threadIdx.x; e < nb * 3 * M; e += blockDim.x) {
        const int b = e / (3 * M), r = e % (3 * M), j = r / 3, c = r % 3;
        sv[e] = v[(size_t)(j0 + j) * n3 + 3 * (b0 + b) + c];
    }
    __syncthreads();
    const int k = blockIdx.y * blockDim.x + threadIdx.x;
    if (k >= nk) return;
    const KVec kv = kvec[k];
    double acc[6 * M];
#pragma unroll
    for (int q = 0; q < 6 * M; ++q) acc[q] = 0.0;
    for (int b = 0; b < nb; ++b) {
        const double2 e = kphase(kv, stab + b * 3 * nm1, nm1);
#pragma unroll
        for (int j = 0; j < M; ++j)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double x = sv[b * 3 * M + 3 * j + c];
                acc[6 * j + c] += e.x * x;
                acc[6 * j + 3 + c] += e.y * x;
            }
    }
    double *o = sfpart + (size_t)chunk * 6 * max_rhs * nk;
#pragma unroll
    for (int j = 0; j < M; ++j)
#pragma unroll
        for (int q = 0; q < 6; ++q) o[(size_t)(6 * (j0 + j) + q) * nk + k] = acc[6 * j + q];
}

void launch_structure_factors(const Ctx &c, const double *v, int m, hipStream_t s)
{
    const int nm1 = c.nmax + 1;
    for (int j0 = 0; j0 < m;) {
        const int mc = (m - j0) >= 4 ? 4 : (m - j0) >= 2 ? 2 : 1;
        const dim3 g(c.nsfc, (c.nk + 255) / 256), b(256);
        const size_t lds = sizeof(double) * (2 * SF_CHUNK * 3 * nm1 + SF_CHUNK * 3 * mc);
        if (mc == 4)
            hipLaunchKernelGGL(k_structure_factors<4>, g, b, lds, s, c.N, c.n3, c.nk, c.nmax,
                               c.kvec, c.etab, v, j0, c.rhs_cap, c.sfpart);
        else if (mc == 2)
            hipLaunchKernelGGL(k_structure_factors<2>, g, b, lds, s, c.N, c.n3, c.nk, c.nmax,
                               c.kvec, c.etab, v, j0, c.rhs_cap, c.sfpart);
        else
            hipLaunchKernelGGL(k_structure_factors<1>, g, b, lds, s, c.N, c.n3, c.nk, c.nmax,
                               c.kvec, c.etab, v, j0, c.rhs_cap, c.sfpart);
        j0 += mc;
    }
}

// Sum the chunk partials in chunk order and apply the reciprocal kernel:
//   Tc_k = 2 m(k) (I - khat khat) C_k,  Ts_k = 2 m(k) (I - khat khat) S_k.
// Block (64 wave vectors) x (4 chunk lanes); grid (k-blocks, m).
__global__ __launch_bounds__(256) void k_sf_reduce(int nk, int nsfc, int max_rhs,
                                                   const KCoef *__restrict__ kcoef,
                                                   const double *__restrict__ sfpart,
                                                   double *__restrict__ tk)
{
    __shared__ double red[4][6][64];
    const int kx = threadIdx.x & 63, q = threadIdx.x >> 6;
    const int k = blockIdx.x * 64 + kx;
    const int j = blockIdx.y;
    double s[6] = {0, 0, 0, 0, 0, 0};
    if (k < nk) {
        for (int ch = q; ch < nsfc; ch += 4) {
            const double *o = sfpart + (size_t)ch * 6 * max_rhs * nk + (size_t)6 * j * nk + k;
#pragma unroll
            for (int c = 0; c < 6; ++c) s[c] += o[(size_t)c * nk];
        }
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) red[q][c][kx] = s[c];
    __syncthreads();
    if (q != 0 || k >= nk) return;
    double t[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) t[c] = ((red[0][c][kx] + red[1][c][kx]) + red[2][c][kx]) + red[3][c][kx];
    const KCoef kc = kcoef[k];
    const double hc = kc.hx * t[0] + kc.hy * t[1] + kc.hz * t[2];
    const double hs = kc.hx * t[3] + kc.hy * t[4] + kc.hz * t[5];
    double *o = tk + (size_t)6 * j * nk + k;
    o[0 * (size_t)nk] = kc.w * (t[0] - kc.hx * hc);
    o[1 * (size_t)nk] = kc.w * (t[1] - kc.hy * hc);
    o[2 * (size_t)nk] = kc.w * (t[2] - kc.hz * hc);
    o[3 * (size_t)nk] = kc.w * (t[3] - kc.hx * hs);
    o[4 * (size_t)nk] = kc.w * (t[4] - kc.hy * hs);
    o[5 * (size_t)nk] = kc.w * (t[5] - kc.hz * hs);
}

void launch_sf_reduce(const Ctx &c, int m, hipStream_t s)
{
    hipLaunchKernelGGL(k_sf_reduce, dim3((c.nk + 63) / 64, m), dim3(256), 0, s, c.nk, c.nsfc,
                       c.rhs_cap, c.kcoef, c.sfpart, c.tk);
}

// ------------------------------------------------------------------ SYMV
// Element types of the stored tiles.  Each lane of a 16-lane row group owns
// 12 fixed columns of the 192-column tile row and loads them with 16-byte
// (or 8-byte) vector loads that are contiguous across the row group.
template <typename T> struct TileT;
template <> struct TileT<double> {
    using acc_t = double;
    __device__ static int col(int q, int e) { return 32 * (e >> 1) + 2 * q + (e & 1); }
    __device__ static void load(const double *row, int q, acc_t a[12])
    {
#pragma unroll
        for (int s = 0; s < 6; ++s) {
            const double2 v = *reinterpret_cast<const double2 *>(row + 32 * s + 2 * q);
            a[2 * s] = v.x;
            a[2 * s + 1] = v.y;
        }
    }
};
template <> struct TileT<float> {
    using acc_t = float;
    __device__ static int col(int q, int e) { return 64 * (e >> 2) + 4 * q + (e & 3); }
    __device__ static void load(const float *row, int q, acc_t a[12])
    {
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const float4 v = *reinterpret_cast<const float4 *>(row + 64 * s + 4 * q);
            a[4 * s] = v.x;
            a[4 * s + 1] = v.y;
            a[4 * s + 2] = v.z;
            a[4 * s + 3] = v.w;
        }
    }
};
template <> struct TileT<uint16_t> {
    using acc_t = float;
    __device__ static int col(int q, int e) { return e < 8 ? 8 * q + e : 128 + 4 * q + (e - 8); }
    __device__ static float bf(uint32_t w, int hi)
    {
        return __uint_as_float(hi ? (w & 0xFFFF0000u) : (w << 16));
    }
    __device__ static void load(const uint16_t *row, int q, acc_t a[12])
    {
        const uint4 v = *reinterpret_cast<const uint4 *>(row + 8 * q);
        const uint2 u = *reinterpret_cast<const uint2 *>(row + 128 + 4 * q);
        a[0] = bf(v.x, 0); a[1] = bf(v.x, 1);
        a[2] = bf(v.y, 0); a[3] = bf(v.y, 1);
        a[4] = bf(v.z, 0); a[5] = bf(v.z, 1);
        a[6] = bf(v.w, 0); a[7] = bf(v.w, 1);
        a[8] = bf(u.x, 0); a[9] = bf(u.x, 1);
        a[10] = bf(u.y, 0); a[11] = bf(u.y, 1);
    }
};

template <typename A> __device__ inline A sum16(A x)
{
#pragma unroll
    for (int o = 8; o >= 1; o >>= 1) x += __shfl_xor(x, o, 16);
    return x;
}

// One workgroup (4 waves) per stored tile (I, J).  Wave w, row group g
// (16 lanes), lane q: rows r = 16 it + 4 w + g, it = 0..11.  Row sums give
// A_IJ x_J -> part[J][j][rows of I]; column sums (off-diagonal tiles only)
// give A_IJ^T x_I -> part[I][j][rows of J].
template <typename T, int M>
__global__ __launch_bounds__(256) void k_symv(int n3, int n3pad, int max_rhs,
                                              const int2 *__restrict__ tile_ij,
                                              const T *__restrict__ tiles,
                                              const double *__restrict__ v,
                                              double *__restrict__ part)
{
    using A = typename TileT<T>::acc_t;
    __shared__ A sx[M][TS];
    __shared__ double scol[4][M][TS];
    const int t = blockIdx.x;
    const int2 ij = tile_ij[t];
    const int I = ij.x, J = ij.y;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane >> 4, q = lane & 15;
    for (int e = threadIdx.x; e < M * TS; e += blockDim.x) {
        const int j = e / TS, r = e % TS, row = I * TS + r;
        sx[j][r] = row < n3 ? (A)v[(size_t)j * n3 + row] : (A)0;
    }
    A xj[M][12];
#pragma unroll
    for (int j = 0; j < M; ++j)
#pragma unroll
        for (int e = 0; e < 12; ++e) {
            const int col = J * TS + TileT<T>::col(q, e);
            xj[j][e] = col < n3 ? (A)v[(size_t)j * n3 + col] : (A)0;
        }
    A cacc[M][12];
#pragma unroll
    for (int j = 0; j < M; ++j)
#pragma unroll
        for (int e = 0; e < 12; ++e) cacc[j][e] = (A)0;
    __syncthreads();
    const T *tile = tiles + (size_t)t * TILE_ELEMS;
    const bool offd = I != J;
#pragma unroll 4
    for (int it = 0; it < TS / 16; ++it) {
        const int r = 16 * it + 4 * w + g;
        A a[12];
        TileT<T>::load(tile + (size_t)r * TS, q, a);
#pragma unroll
        for (int j = 0; j < M; ++j) {
            A rs = (A)0;
#pragma unroll
            for (int e = 0; e < 12; ++e) rs += a[e] * xj[j][e];
            rs = sum16(rs);
            if (q == 0) part[((size_t)J * max_rhs + j) * n3pad + I * TS + r] = (double)rs;
            if (offd) {
                const A xr = sx[j][r];
#pragma unroll
                for (int e = 0; e < 12; ++e) cacc[j][e] += a[e] * xr;
            }
        }
    }
    if (!offd) return;
    // combine the 4 row groups of a wave, then the 4 waves through LDS
#pragma unroll
    for (int j = 0; j < M; ++j)
#pragma unroll
        for (int e = 0; e < 12; ++e) {
            double s = (double)cacc[j][e];
            s += __shfl_xor(s, 16);
            s += __shfl_xor(s, 32);
            if (g == 0) scol[w][j][TileT<T>::col(q, e)] = s;
        }
    __syncthreads();
    for (int e = threadIdx.x; e < M * TS; e += blockDim.x) {
        const int j = e / TS, cidx = e % TS;
        const double s = ((scol[0][j][cidx] + scol[1][j][cidx]) + scol[2][j][cidx]) + scol[3][j][cidx];
        part[((size_t)I * max_rhs + j) * n3pad + J * TS + cidx] = s;
    }
}

template <typename T>
static void symv_typed(const Ctx &c, const T *tiles, const double *v, int m, hipStream_t s)
{
    for (int j0 = 0; j0 < m;) {
        const int mc = (m - j0) >= 4 ? 4 : (m - j0) >= 2 ? 2 : 1;
        double *part = c.part + (size_t)j0 * c.n3pad;
        const double *vj = v + (size_t)j0 * c.n3;
        const dim3 g(c.ntiles), b(256);
        if (mc == 4)
            hipLaunchKernelGGL((k_symv<T, 4>), g, b, 0, s, c.n3, c.n3pad, c.rhs_cap, c.tile_ij,
                               tiles, vj, part);
        else if (mc == 2)
            hipLaunchKernelGGL((k_symv<T, 2>), g, b, 0, s, c.n3, c.n3pad, c.rhs_cap, c.tile_ij,
                               tiles, vj, part);
        else
            hipLaunchKernelGGL((k_symv<T, 1>), g, b, 0, s, c.n3, c.n3pad, c.rhs_cap, c.tile_ij,
                               tiles, vj, part);
        j0 += mc;
    }
}

void launch_symv(const Ctx &c, int prec, const double *v, int m, hipStream_t s)
{
    if (prec == RPY_PREC_F32)
        symv_typed<float>(c, c.d32, v, m, s);
    else if (prec == RPY_PREC_BF16)
        symv_typed<uint16_t>(c, c.d16, v, m, s);
    else
        symv_typed<double>(c, c.d64, v, m, s);
}

// ------------------------------------------------------------- finalize
// 16 beads per workgroup, 16 lanes per bead.  Lane q of bead nu sums the
// tile partials K = q, q+16, ... and the reciprocal terms k = q, q+16, ...:
//   y = sum_K part[K] + sum_k cos(k.r_nu) Tc_k + sin(k.r_nu) Ts_k,
// the 16 lanes are combined, then the epilogue of `mode` writes the result.
template <int M>
__global__ __launch_bounds__(256) void k_finalize(int N, int n3, int n3pad, int nbt, int nk,
                                                  int nmax, int max_rhs,
                                                  const KVec *__restrict__ kvec,
                                                  const double2 *__restrict__ etab,
                                                  const double *__restrict__ part,
                                                  const double *__restrict__ tk, int j0,
                                                  FinArgs f)
{
    const int nm1 = nmax + 1;
    extern __shared__ double2 stab[];   // [FIN_BEADS][3*nm1]
    const int b0 = blockIdx.x * FIN_BEADS;
    const int nb = min(FIN_BEADS, N - b0);
    for (int e = threadIdx.x; e < nb * 3 * nm1; e += blockDim.x)
        stab[e] = etab[(size_t)b0 * 3 * nm1 + e];
    __syncthreads();
    const int bl = threadIdx.x >> 4, q = threadIdx.x & 15;
    const int nu = b0 + bl;
    const bool live = bl < nb;
    double y[M][3];
#pragma unroll
    for (int j = 0; j < M; ++j) y[j][0] = y[j][1] = y[j][2] = 0.0;
    if (live) {
        for (int K = q; K < nbt; K += 16) {
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const double *pp = part + ((size_t)K * max_rhs + j0 + j) * n3pad + 3 * nu;
                y[j][0] += pp[0];
                y[j][1] += pp[1];
                y[j][2] += pp[2];
            }
        }
        const double2 *tab = stab + bl * 3 * nm1;
        for (int k = q; k < nk; k += 16) {
            const double2 e = kphase(kvec[k], tab, nm1);
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const double *tt = tk + (size_t)6 * (j0 + j) * nk + k;
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    y[j][c] += e.x * tt[(size_t)c * nk] + e.y * tt[(size_t)(3 + c) * nk];
            }
        }
    }
#pragma unroll
    for (int j = 0; j < M; ++j)
#pragma unroll
        for (int c = 0; c < 3; ++c) y[j][c] = sum16(y[j][c]);
    if (!live) return;
    const double ya = f.scal ? f.scal[2] : 0.0, yb = f.scal ? f.scal[3] : 0.0;
#pragma unroll
    for (int j = 0; j < M; ++j)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if ((3 * j + c) % 16 != q) continue;
            const size_t o = (size_t)(j0 + j) * n3 + 3 * nu + c;
            if (f.mode == FIN_APPLY) {
                f.vout[o] = y[j][c];
            } else if (f.mode == FIN_CHEB_FIRST) {
                const double v0 = f.vprev[o];
                const double v1 = ya * y[j][c] - yb * v0;
                f.vout[o] = v1;
                f.acc[o] = 0.5 * f.scal[8] * v0 + f.scal[9] * v1;
                if (f.dv) f.dv[o] = y[j][c];
            } else {
                const double vp = 2.0 * (ya * y[j][c] - yb * f.vprev[o]) - f.vprev2[o];
                f.vout[o] = vp;
                f.acc[o] += f.scal[8 + f.p] * vp;
            }
        }
}

void launch_finalize(const Ctx &c, const FinArgs &f, hipStream_t s)
{
    const size_t lds = sizeof(double2) * FIN_BEADS * 3 * (c.nmax + 1);
    const dim3 g((c.N + FIN_BEADS - 1) / FIN_BEADS), b(256);
    for (int j0 = 0; j0 < f.m;) {
        const int mc = (f.m - j0) >= 4 ? 4 : (f.m - j0) >= 2 ? 2 : 1;
        if (mc == 4)
            hipLaunchKernelGGL(k_finalize<4>, g, b, lds, s, c.N, c.n3, c.n3pad, c.nbt, c.nk,
                               c.nmax, c.rhs_cap, c.kvec, c.etab, c.part, c.tk, j0, f);
        else if (mc == 2)
            hipLaunchKernelGGL(k_finalize<2>, g, b, lds, s, c.N, c.n3, c.n3pad, c.nbt, c.nk,
                               c.nmax, c.rhs_cap, c.kvec, c.etab, c.part, c.tk, j0, f);
        else
            hipLaunchKernelGGL(k_finalize<1>, g, b, lds, s, c.N, c.n3, c.n3pad, c.nbt, c.nk,
                               c.nmax, c.rhs_cap, c.kvec, c.etab, c.part, c.tk, j0, f);
        j0 += mc;
    }
}

// ------------------------------------------------- Chebyshev coefficients
// scal[0] = d_min, scal[1] = d_max, scal[2] = 2/(d_max - d_min),
// scal[3] = (d_max + d_min)/(d_max - d_min), scal[8 + p] = c_p with
//   c_p = (2/n) sum_{j=1..n} sqrt(h x_j + m) cos(p theta_j),
//   theta_j = pi (j - 1/2)/n, x_j = cos theta_j, h = (d_max-d_min)/2, m = (d_max+d_min)/2.
// rule = RPY_BOUNDS_PAPER derives the interval from du = D.U+ first.
__global__ __launch_bounds__(256) void k_cheb_coeffs(int nbeads, int n, int rule, double C,
                                                     double dmin, double dmax,
                                                     const double *__restrict__ du,
                                                     double *__restrict__ scal)
{
    __shared__ double red[256];
    __shared__ double bounds[2];
    if (rule == RPY_BOUNDS_PAPER) {
        const int n3 = 3 * nbeads;
        double s = 0.0;
        for (int i = threadIdx.x; i < n3; i += blockDim.x) s += du[i];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const double lf = red[0] / n3;
            const double np6 = pow((double)nbeads, 0.6);
            const double lmax = 0.35 * np6 * lf;
            bounds[0] = lmax / (C * np6);
            bounds[1] = lmax;
        }
    } else if (threadIdx.x == 0) {
        bounds[0] = dmin;
        bounds[1] = dmax;
    }
    __syncthreads();
    const double lo = bounds[0], hi = bounds[1];
    const double h = 0.5 * (hi - lo), mid = 0.5 * (hi + lo);
    for (int p = threadIdx.x; p < n; p += blockDim.x) {
        double s = 0.0;
        for (int j = 1; j <= n; ++j) {
            const double u = (j - 0.5) / n;
            const double fx = sqrt(h * cospi(u) + mid);
            s += fx * cospi(p * u);
        }
        scal[8 + p] = 2.0 * s / n;
    }
    if (threadIdx.x == 0) {
        scal[0] = lo;
        scal[1] = hi;
        scal[2] = 2.0 / (hi - lo);
        scal[3] = (hi + lo) / (hi - lo);
    }
}

void launch_cheb_coeffs(const Ctx &c, int n_cheb, int rule, double C, double dmin, double dmax,
                        const double *du, hipStream_t s)
{
    hipLaunchKernelGGL(k_cheb_coeffs, dim3(1), dim3(256), 0, s, c.N, n_cheb, rule, C, dmin,
                       dmax, du, c.scal);
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
