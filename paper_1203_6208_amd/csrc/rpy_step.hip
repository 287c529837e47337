// rpy_step.hip -- forces, noise, Euler update and chain observables of the
// Brownian-dynamics step (arXiv:1203.6208, section "Governing equation" and
// section "Testing and verification").
#include "rpy_internal.h"

namespace rpy {

// Hookean springs: F_mu = Q_mu - Q_{mu-1}, Q_mu = r_{mu+1} - r_mu within a
// chain (unwrapped positions).  Overwrites F.
__global__ void k_springs(int N, int bpc, const double *__restrict__ pos, double *__restrict__ F)
{
    const int mu = blockIdx.x * blockDim.x + threadIdx.x;
    if (mu >= N) return;
    const int b = mu % bpc;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        double f = 0.0;
        if (b + 1 < bpc) f += pos[3 * (mu + 1) + i] - pos[3 * mu + i];
        if (b > 0) f -= pos[3 * mu + i] - pos[3 * (mu - 1) + i];
        F[3 * mu + i] = f;
    }
}

void launch_spring_forces(const Ctx &c, const double *pos, double *F, hipStream_t s)
{
    hipLaunchKernelGGL(k_springs, dim3((c.N + 255) / 256), dim3(256), 0, s, c.N, c.bpc, pos, F);
}

// --------------------------------------------------------------- cell list
// Cells of side >= rcut (ncell per axis, at least 3 so the 27-cell stencil
// visits distinct cells); beads sorted by cell, by index inside a cell.
__device__ inline int cell_of(const double *rt, int nu, double L, int nc)
{
    int cx = (int)(rt[3 * nu] / L * nc), cy = (int)(rt[3 * nu + 1] / L * nc),
        cz = (int)(rt[3 * nu + 2] / L * nc);
    cx = min(max(cx, 0), nc - 1);
    cy = min(max(cy, 0), nc - 1);
    cz = min(max(cz, 0), nc - 1);
    return (cz * nc + cy) * nc + cx;
}

__global__ void k_cell_zero(int n, int *a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0;
}

__global__ void k_cell_count(int N, double L, int nc, const double *__restrict__ rt, int *count)
{
    const int nu = blockIdx.x * blockDim.x + threadIdx.x;
    if (nu >= N) return;
    atomicAdd(&count[cell_of(rt, nu, L, nc)], 1);
}

// Exclusive scan of the counts (one workgroup, Hillis-Steele over the
// per-thread partial sums), start[ncells] = N; the counts are reset to serve
// as insertion cursors.
__global__ __launch_bounds__(1024) void k_cell_scan(int ncells, int *count, int *start)
{
    __shared__ int part[2][1024];
    const int tid = threadIdx.x;
    const int per = (ncells + 1023) / 1024;
    const int lo = min(tid * per, ncells), hi = min(lo + per, ncells);
    int s = 0;
    for (int i = lo; i < hi; ++i) s += count[i];
    int cur = 0;
    part[0][tid] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int v = part[cur][tid] + (tid >= off ? part[cur][tid - off] : 0);
        part[cur ^ 1][tid] = v;
        cur ^= 1;
        __syncthreads();
    }
    int run = part[cur][tid] - s;   // exclusive prefix
    for (int i = lo; i < hi; ++i) {
        start[i] = run;
        run += count[i];
        count[i] = 0;
    }
    if (tid == 1023) start[ncells] = run;
}

__global__ void k_cell_fill(int N, double L, int nc, const double *__restrict__ rt,
                            const int *__restrict__ start, int *cursor, int *beads)
{
    const int nu = blockIdx.x * blockDim.x + threadIdx.x;
    if (nu >= N) return;
    const int c = cell_of(rt, nu, L, nc);
    const int slot = atomicAdd(&cursor[c], 1);
    beads[start[c] + slot] = nu;
}

// One workgroup per cell: order the cell's beads by index (each entry's rank
// among the distinct indices) so that every later sum over a cell runs in a
// fixed order.  Cells above SORT_CAP entries (more than a quarter of a
// million beads in 27 cells) fall back to a serial sort.
constexpr int SORT_CAP = 8192;
__global__ __launch_bounds__(256) void k_cell_sort(const int *__restrict__ start, int *beads)
{
    __shared__ int sb[SORT_CAP];
    const int c = blockIdx.x;
    const int lo = start[c], n = start[c + 1] - lo;
    if (n <= 1) return;
    if (n > SORT_CAP) {
        if (threadIdx.x == 0) {
            for (int i = lo + 1; i < lo + n; ++i) {
                const int v = beads[i];
                int j = i - 1;
                while (j >= lo && beads[j] > v) {
                    beads[j + 1] = beads[j];
                    --j;
                }
                beads[j + 1] = v;
            }
        }
        return;
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) sb[i] = beads[lo + i];
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int v = sb[i];
        int r = 0;
        for (int j = 0; j < n; ++j) r += sb[j] < v;
        beads[lo + r] = v;
    }
}

// Cell list of N wrapped positions rt into nc^3 cells: start [nc^3 + 1] (and a
// cursor area of nc^3 more ints after it), beads [N] sorted by cell, by index
// inside a cell.
void launch_cell_list_into(int N, double L, int nc, const double *rt, int *start, int *beads,
                           hipStream_t s)
{
    if (nc < 3) return;
    const int ncells = nc * nc * nc;
    int *count = start + ncells + 1;  // cursor area
    hipLaunchKernelGGL(k_cell_zero, dim3((ncells + 255) / 256), dim3(256), 0, s, ncells, count);
    hipLaunchKernelGGL(k_cell_count, dim3((N + 255) / 256), dim3(256), 0, s, N, L, nc, rt, count);
    hipLaunchKernelGGL(k_cell_scan, dim3(1), dim3(1024), 0, s, ncells, count, start);
    hipLaunchKernelGGL(k_cell_fill, dim3((N + 255) / 256), dim3(256), 0, s, N, L, nc, rt, start,
                       count, beads);
    hipLaunchKernelGGL(k_cell_sort, dim3(ncells), dim3(256), 0, s, start, beads);
}

void launch_cell_list(const Ctx &c, const double *rt, double rcut, hipStream_t s)
{
    (void)rcut;
    launch_cell_list_into(c.N, c.L, c.ncell, rt, c.cell_start, c.cell_beads, s);
}

// Narrow-Gaussian excluded volume, minimum image (rcut < L/2):
//   F_nu += (z*/d*^5) d exp(-|d|^2 / (2 d*^2)), d = r_nu - r_mu, |d| <= rcut.
// One workgroup per home cell.  The neighbour-cell offsets, the home beads
// (in batches of 4 EV_HMAX) and the beads of the 27 surrounding cells (in
// batches of EV_CAP) are staged in LDS by parallel loads; each wave then
// takes home beads in turn and its 64 lanes split the candidates; a fixed
// xor tree combines the lanes.
// VJP: the transpose of the force Jacobian applied to gF instead,
//   out_nu += sum_mu J(d) (gF_nu - gF_mu),
//   J(d) = (z*/d*^5) exp(-|d|^2 / (2 d*^2)) (I - d d^T / d*^2)
// (J is the d-derivative of the pair force, symmetric and even in d).
constexpr int EV_CAP = 1024;
constexpr int EV_HMAX = 8;   // home beads per wave per batch
template <bool VJP>
__global__ __launch_bounds__(256) void k_ev_cells(double L, int nc, const double *__restrict__ rt,
                                                  const int *__restrict__ start,
                                                  const int *__restrict__ beads, double pref,
                                                  double inv2d2, double rcut2,
                                                  const double *__restrict__ gF,
                                                  double *__restrict__ F)
{
    __shared__ double sx[EV_CAP], sy[EV_CAP], sz[EV_CAP];
    __shared__ int sid[EV_CAP];
    __shared__ double hx[4 * EV_HMAX], hy[4 * EV_HMAX], hz[4 * EV_HMAX];
    __shared__ int hid[4 * EV_HMAX];
    __shared__ double sg[VJP ? 3 * EV_CAP : 1];        // gF of the staged candidates
    __shared__ double hg[VJP ? 3 * 4 * EV_HMAX : 1];   // gF of the home beads
    __shared__ int nbr_start[27];
    __shared__ int nbr_off[28];
    const int c = blockIdx.x;
    const int cx = c % nc, cy = (c / nc) % nc, cz = c / (nc * nc);
    if (threadIdx.x < 27) {
        const int q = threadIdx.x;
        const int ox = q % 3 - 1, oy = (q / 3) % 3 - 1, oz = q / 9 - 1;
        const int ex = (cx + ox + nc) % nc, ey = (cy + oy + nc) % nc, ez = (cz + oz + nc) % nc;
        const int cc = (ez * nc + ey) * nc + ex;
        const int st = start[cc];
        nbr_start[q] = st;
        nbr_off[q + 1] = start[cc + 1] - st;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        nbr_off[0] = 0;
        for (int q = 0; q < 27; ++q) nbr_off[q + 1] += nbr_off[q];
    }
    __syncthreads();
    const int hlo = start[c], nh = start[c + 1] - hlo;
    const int total = nbr_off[27];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const double invL = 1.0 / L;
    for (int h0 = 0; h0 < nh; h0 += 4 * EV_HMAX) {
        const int nhb = min(4 * EV_HMAX, nh - h0);
        if (threadIdx.x < nhb) {
            const int nu = beads[hlo + h0 + threadIdx.x];
            hid[threadIdx.x] = nu;
            hx[threadIdx.x] = rt[3 * nu];
            hy[threadIdx.x] = rt[3 * nu + 1];
            hz[threadIdx.x] = rt[3 * nu + 2];
            if (VJP)
                for (int c = 0; c < 3; ++c) hg[3 * threadIdx.x + c] = gF[3 * nu + c];
        }
        double acc[EV_HMAX][3];
#pragma unroll
        for (int i = 0; i < EV_HMAX; ++i) acc[i][0] = acc[i][1] = acc[i][2] = 0.0;
        for (int b0 = 0; b0 < total; b0 += EV_CAP) {
            const int nb = min(EV_CAP, total - b0);
            __syncthreads();
            for (int e = threadIdx.x; e < nb; e += blockDim.x) {
                const int g = b0 + e;
                int q = 0;
                while (nbr_off[q + 1] <= g) ++q;
                const int mu = beads[nbr_start[q] + (g - nbr_off[q])];
                sid[e] = mu;
                sx[e] = rt[3 * mu];
                sy[e] = rt[3 * mu + 1];
                sz[e] = rt[3 * mu + 2];
                if (VJP)
                    for (int c = 0; c < 3; ++c) sg[3 * e + c] = gF[3 * mu + c];
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < EV_HMAX; ++i) {
                const int li = 4 * i + w;
                if (li < nhb) {
                    const int nu = hid[li];
                    const double x = hx[li], y = hy[li], z = hz[li];
                    for (int e = lane; e < nb; e += 64) {
                        if (sid[e] == nu) continue;
                        double dx = x - sx[e], dy = y - sy[e], dz = z - sz[e];
                        dx -= L * rint(dx * invL);
                        dy -= L * rint(dy * invL);
                        dz -= L * rint(dz * invL);
                        const double r2 = dx * dx + dy * dy + dz * dz;
                        if (r2 > rcut2) continue;
                        const double wgt = pref * exp(-r2 * inv2d2);
                        if (VJP) {
                            const double ux = hg[3 * li] - sg[3 * e];
                            const double uy = hg[3 * li + 1] - sg[3 * e + 1];
                            const double uz = hg[3 * li + 2] - sg[3 * e + 2];
                            const double du = (dx * ux + dy * uy + dz * uz) * (2.0 * inv2d2);
                            acc[i][0] += wgt * (ux - dx * du);
                            acc[i][1] += wgt * (uy - dy * du);
                            acc[i][2] += wgt * (uz - dz * du);
                        } else {
                            acc[i][0] += wgt * dx;
                            acc[i][1] += wgt * dy;
                            acc[i][2] += wgt * dz;
                        }
                    }
                }
            }
        }
#pragma unroll
        for (int i = 0; i < EV_HMAX; ++i) {
            const int li = 4 * i + w;
            double f0 = acc[i][0], f1 = acc[i][1], f2 = acc[i][2];
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) {
                f0 += __shfl_xor(f0, o);
                f1 += __shfl_xor(f1, o);
                f2 += __shfl_xor(f2, o);
            }
            if (li < nhb && lane == 0) {
                const int nu = hid[li];
                F[3 * nu] += f0;
                F[3 * nu + 1] += f1;
                F[3 * nu + 2] += f2;
            }
        }
        __syncthreads();   // hid/hx are rewritten by the next home batch
    }
}

// Without a cell list (fewer than 3 cells per side): all pairs per bead.
template <bool VJP>
__global__ void k_ev_pairs(int N, double L, const double *__restrict__ rt, double pref,
                           double inv2d2, double rcut2, const double *__restrict__ gF,
                           double *__restrict__ F)
{
    const int nu = blockIdx.x * blockDim.x + threadIdx.x;
    if (nu >= N) return;
    const double x = rt[3 * nu], y = rt[3 * nu + 1], z = rt[3 * nu + 2];
    const double invL = 1.0 / L;
    double f0 = 0.0, f1 = 0.0, f2 = 0.0;
    for (int mu = 0; mu < N; ++mu) {
        if (mu == nu) continue;
        double dx = x - rt[3 * mu], dy = y - rt[3 * mu + 1], dz = z - rt[3 * mu + 2];
        dx -= L * rint(dx * invL);
        dy -= L * rint(dy * invL);
        dz -= L * rint(dz * invL);
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 > rcut2) continue;
        const double w = pref * exp(-r2 * inv2d2);
        if (VJP) {
            const double ux = gF[3 * nu] - gF[3 * mu], uy = gF[3 * nu + 1] - gF[3 * mu + 1],
                         uz = gF[3 * nu + 2] - gF[3 * mu + 2];
            const double du = (dx * ux + dy * uy + dz * uz) * (2.0 * inv2d2);
            f0 += w * (ux - dx * du);
            f1 += w * (uy - dy * du);
            f2 += w * (uz - dz * du);
        } else {
            f0 += w * dx;
            f1 += w * dy;
            f2 += w * dz;
        }
    }
    F[3 * nu] += f0;
    F[3 * nu + 1] += f1;
    F[3 * nu + 2] += f2;
}

template <bool VJP>
static void ev_launch(const Ctx &c, const double *rt, double zstar, double dstar, double rcut,
                      const double *gF, double *F, hipStream_t s)
{
    const double d2 = dstar * dstar;
    const double pref = zstar / (d2 * d2 * dstar);
    if (c.ncell >= 3) {
        const int ncells = c.ncell * c.ncell * c.ncell;
        hipLaunchKernelGGL(k_ev_cells<VJP>, dim3(ncells), dim3(256), 0, s, c.L, c.ncell, rt,
                           c.cell_start, c.cell_beads, pref, 1.0 / (2.0 * d2), rcut * rcut, gF,
                           F);
    } else {
        hipLaunchKernelGGL(k_ev_pairs<VJP>, dim3((c.N + 127) / 128), dim3(128), 0, s, c.N, c.L,
                           rt, pref, 1.0 / (2.0 * d2), rcut * rcut, gF, F);
    }
}

void launch_ev_forces(const Ctx &c, const double *rt, double zstar, double dstar, double rcut,
                      double *F, hipStream_t s)
{
    ev_launch<false>(c, rt, zstar, dstar, rcut, nullptr, F, s);
}

void launch_ev_vjp(const Ctx &c, const double *rt, double zstar, double dstar, double rcut,
                   const double *gF, double *gpos, hipStream_t s)
{
    ev_launch<true>(c, rt, zstar, dstar, rcut, gF, gpos, s);
}

// ------------------------------------------------------------------ Philox
// Raw Philox4x32-10 blocks (philox10 in rpy_internal.h).
__global__ void k_philox(const uint32_t *__restrict__ ck, uint32_t *__restrict__ out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t *p = ck + 6 * i;
    const uint4 r = philox10(make_uint4(p[0], p[1], p[2], p[3]), make_uint2(p[4], p[5]));
    out[4 * i] = r.x;
    out[4 * i + 1] = r.y;
    out[4 * i + 2] = r.z;
    out[4 * i + 3] = r.w;
}

void launch_philox(const uint32_t *ck, uint32_t *out, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_philox, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ck, out, n);
}

// Gaussian noise: element e uses block g = e/4, counter (g, step lo, step hi,
// 0x52505942), key (seed lo, seed hi); u = (x + 1/2) 2^-32; Box-Muller
// z0 = rho cos(2 pi u1), z1 = rho sin(2 pi u1), rho = sqrt(-2 ln u0), z2/z3
// from (u2, u3).  Scaled by sqrt(dt).
__global__ void k_noise(double *__restrict__ out, int64_t count, uint64_t seed, uint64_t step,
                        double sdt)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (4 * g >= count) return;
    const uint4 x = philox10(make_uint4((uint32_t)g, (uint32_t)step, (uint32_t)(step >> 32),
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
    for (int j = 0; j < 4; ++j)
        if (4 * g + j < count) out[4 * g + j] = z[j] * sdt;
}

void launch_noise(double *out, int64_t count, uint64_t seed, uint64_t step, double dt,
                  hipStream_t s)
{
    const int64_t ng = (count + 3) / 4;
    hipLaunchKernelGGL(k_noise, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, s, out, count,
                       seed, step, sqrt(dt));
}

// Euler-Maruyama update r += (dt/4) D.F + dS/sqrt(2) (eq. sde, kappa = 0).
// The first Chebyshev step from a product computed before the coefficients
// (bd_step folds D.dW into its drift product): with y = D.V_0,
//   V_1 = ya y - yb V_0,  acc = (c_0/2) V_0 + c_1 V_1,  dv = y
// (eq. cheb2; the same operations as the EPI_CHEB_FIRST epilogue).
__global__ void k_cheb_first(int n3, const double *__restrict__ y, const double *__restrict__ v0,
                             const double *__restrict__ scal, double *__restrict__ v1,
                             double *__restrict__ acc, double *__restrict__ dv)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n3) return;
    const double ya = scal[2], yb = scal[3];
    const double yy = y[i], a = v0[i];
    const double b = ya * yy - yb * a;
    v1[i] = b;
    acc[i] = 0.5 * scal[8] * a + scal[9] * b;
    dv[i] = yy;
}

void launch_cheb_first(const Ctx &c, const double *y, const double *v0, double *v1, double *acc,
                       double *dv, hipStream_t s)
{
    hipLaunchKernelGGL(k_cheb_first, dim3((c.n3 + 255) / 256), dim3(256), 0, s, c.n3, y, v0,
                       c.scal, v1, acc, dv);
}

__global__ void k_euler(int n3, double *__restrict__ pos, double dt4,
                        const double *__restrict__ ud, const double *__restrict__ ds)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n3) return;
    pos[i] = pos[i] + dt4 * ud[i] + ds[i] / 1.4142135623730951;
}

void launch_euler(const Ctx &c, double *pos, double dt, const double *ud, const double *ds,
                  hipStream_t s)
{
    hipLaunchKernelGGL(k_euler, dim3((c.n3 + 255) / 256), dim3(256), 0, s, c.n3, pos, dt / 4.0,
                       ud, ds);
}

// One thread per chain: R_e^2 and R_g^2 = mean |r - r_cm|^2.
__global__ void k_observables(int nchains, int bpc, const double *__restrict__ pos,
                              double *__restrict__ re2, double *__restrict__ rg2)
{
    const int ch = blockIdx.x * blockDim.x + threadIdx.x;
    if (ch >= nchains) return;
    const double *x = pos + (size_t)3 * ch * bpc;
    double cm[3] = {0, 0, 0};
    for (int b = 0; b < bpc; ++b)
        for (int i = 0; i < 3; ++i) cm[i] += x[3 * b + i];
    for (int i = 0; i < 3; ++i) cm[i] /= bpc;
    double g = 0.0;
    for (int b = 0; b < bpc; ++b)
        for (int i = 0; i < 3; ++i) {
            const double d = x[3 * b + i] - cm[i];
            g += d * d;
        }
    double e = 0.0;
    for (int i = 0; i < 3; ++i) {
        const double d = x[3 * (bpc - 1) + i] - x[i];
        e += d * d;
    }
    re2[ch] = e;
    rg2[ch] = g / bpc;
}

void launch_observables(const Ctx &c, const double *pos, double *re2, double *rg2,
                        hipStream_t s)
{
    hipLaunchKernelGGL(k_observables, dim3((c.nchains + 127) / 128), dim3(128), 0, s, c.nchains,
                       c.bpc, pos, re2, rg2);
}

}  // namespace rpy
