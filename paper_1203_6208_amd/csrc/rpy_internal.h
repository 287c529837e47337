// rpy_internal.h -- internal declarations of librpy (gfx950).
//
// Storage of the real-space diffusion matrix: the 3N x 3N matrix is cut into
// square tiles of TB = 64 beads (TS = 192 rows/columns).  Only the tiles
// (I, J) with I <= J are stored (D is symmetric), contiguous, in the order
// t = I*nbt - I*(I-1)/2 + (J - I).  Beads past N have zero entries.
//   FP64 tiles (d64): every 3 x 3 bead-pair block of D is itself symmetric
//   (each pair term is a I + b rhat rhat), so a tile keeps 6 entries per bead
//   pair, as planes: d64[t][i][c][j] (TILE6 doubles), i, j the beads of I and
//   J within the tile, c = xx, xy, xz, yy, yz, zz.
//   FP32 / BF16 tiles: packed the same way (p32, p16); every product, the
//   matrix-core block product included, reads these packed planes.
// A product y = D.x reads every stored tile once and produces both A_IJ x_J
// (rows of I) and A_IJ^T x_I (rows of J); the partial results land in
// part[K][j][row] so that row r of y is the fixed-order sum over K of
// part[K][j][r] (K = the tile column the contribution came from).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rpy.h"

#define RPY_HD __host__ __device__

namespace rpy {

constexpr int TB = 64;          // beads per tile side
constexpr int TS = 3 * TB;      // matrix rows per tile side
constexpr int TILE_ELEMS = TS * TS;
constexpr int TILE6 = 6 * TB * TB;   // packed FP64 tile: 6 planes per bead row
// Tile arrays up to TILE_CACHE_BYTES are read with allocating loads and stay
// in the 256 MB Infinity Cache from one product to the next (measured at
// N = 4000: FP32 tiles, 192 MB, 44.1 -> 39.2 us; BF16, 96 MB, 33.9 -> 30.6
// us).  Larger arrays stream with non-temporal loads in stored order, which
// keeps the rest of the product's data (partials, vectors, T_k) cached: for
// the FP64 tiles at N = 4000 (384 MB) allocating loads with the tile order
// reversed on every other launch read part of the array from the cache, but
// the step runs faster without them (254.0 against 251.5 steps/s).
constexpr size_t TILE_CACHE_BYTES = (size_t)200 << 20;
constexpr int NSER = 20;        // terms of the small-r series of S(r)
constexpr double XSER = 0.75;   // use the series for alpha*r below this
constexpr int MAX_RHS = 16;
constexpr int MAX_NCHEB = 512;
constexpr int MAX_LANCZOS = 2048;
constexpr int KSLICE = 16;      // wave-vector / tile-column slices of the back-projection
constexpr int SF_BEADS = 64;    // beads per structure-factor partial

// ---------------------------------------------------------------- pair terms
// Constants of the real-space pair kernel.  Passed by value to kernels.
struct PairConst {
    double L, invL;
    double a, alpha;
    double rc, rc2;        // real-space cutoff
    double reach;          // max(rc, 2a): images beyond it contribute nothing
    double a2x4;           // (2a)^2
    double self_coeff;     // 1 - 6 a al/sqrt(pi) + 40 a^3 al^3 / (3 sqrt(pi))
    double A1, A3;         // a*alpha and (a*alpha)^3
    double inv_sqrtpi;
    double inv_A1sq;       // 1 / (a alpha)^2
    double s1[NSER], s2[NSER];  // series of S1, S2 in (alpha r)^2
};

// Real-space Ewald kernel M1 (eq. M1) written in x = alpha r:
//   c1 = erfc(x)(3a/4r + a^3/2r^3)
//        + e^{-x^2}/sqrt(pi) [A1 (3x^2 - 9/2) + A3 (4x^4 - 20x^2 + 14 + 1/x^2)]
//   c2 = erfc(x)(3a/4r - 3a^3/2r^3)
//        + e^{-x^2}/sqrt(pi) [A1 (3/2 - 3x^2) + A3 (-4x^4 + 16x^2 - 2 - 3/x^2)]
RPY_HD inline void m1_coeffs(double r, const PairConst &p, double &c1, double &c2)
{
    const double x = p.alpha * r;
    const double x2 = x * x;
    const double e = erfc(x);
    const double g = exp(-x2) * p.inv_sqrtpi;
    const double ar = p.a * (1.0 / r);
    const double ar3 = ar * ar * ar;
    const double ix2 = ar * ar * p.inv_A1sq;   // 1/x^2 = (a/r)^2 / (a alpha)^2
    c1 = e * (0.75 * ar + 0.5 * ar3)
       + g * (p.A1 * (3.0 * x2 - 4.5) + p.A3 * ((4.0 * x2 - 20.0) * x2 + 14.0 + ix2));
    c2 = e * (0.75 * ar - 1.5 * ar3)
       + g * (p.A1 * (1.5 - 3.0 * x2) + p.A3 * ((16.0 - 4.0 * x2) * x2 - 2.0 - 3.0 * ix2));
}

// Smooth part S = Omega_A - M1 (the piece the reciprocal sum carries), an
// even entire function of x = alpha r.  For x < XSER its power series in x^2
// (coefficients from the series of erf and exp, see make_pair_const); else
//   S1 = A1 [3/4 erf(x)/x - (3x^2 - 9/2) e^{-x^2}/sqrt(pi)]
//      + A3 [1/2 erf(x)/x^3 - (4x^4 - 20x^2 + 14 + 1/x^2) e^{-x^2}/sqrt(pi)]
//   S2 = A1 [3/4 erf(x)/x - (3/2 - 3x^2) e^{-x^2}/sqrt(pi)]
//      + A3 [-3/2 erf(x)/x^3 - (-4x^4 + 16x^2 - 2 - 3/x^2) e^{-x^2}/sqrt(pi)]
RPY_HD inline void smooth_part(double x, const PairConst &p, double &s1, double &s2)
{
    const double x2 = x * x;
    if (x < XSER) {
        double u = p.s1[NSER - 1], v = p.s2[NSER - 1];
        for (int n = NSER - 2; n >= 0; --n) {
            u = u * x2 + p.s1[n];
            v = v * x2 + p.s2[n];
        }
        s1 = u;
        s2 = v;
    } else {
        const double ef = erf(x);
        const double g = exp(-x2) * p.inv_sqrtpi;
        const double ex1 = ef / x, ex3 = ef / (x * x2), ix2 = 1.0 / x2;
        s1 = p.A1 * (0.75 * ex1 - (3.0 * x2 - 4.5) * g)
           + p.A3 * (0.5 * ex3 - ((4.0 * x2 - 20.0) * x2 + 14.0 + ix2) * g);
        s2 = p.A1 * (0.75 * ex1 - (1.5 - 3.0 * x2) * g)
           + p.A3 * (-1.5 * ex3 - ((16.0 - 4.0 * x2) * x2 - 2.0 - 3.0 * ix2) * g);
    }
}

// Contribution of one periodic image d of a pair to the symmetric 3x3
// block b = {xx, xy, xz, yy, yz, zz}:
//   |d| <= rc, |d| >= 2a : M1(d)
//   |d| <= rc, |d| <  2a : M1 + M* = Omega_B - S   (stable at small r)
//   |d| >  rc, |d| <  2a : M* = Omega_B - Omega_A  (eq. cor5)
// The coefficients c1 (of I) and c2 (of rhat rhat) of an image at squared
// distance r2 that contributes (r2 <= rc^2 or r2 < (2a)^2).
RPY_HD inline void image_coeffs(double r2, const PairConst &p, double &c1, double &c2)
{
    const bool in_rc = r2 <= p.rc2;
    const bool ov = r2 < p.a2x4;
    const double r = sqrt(r2);
    if (!ov) {
        m1_coeffs(r, p, c1, c2);
    } else {
        const double xa = r / p.a;
        const double ob1 = 1.0 - 0.28125 * xa;   // 9/32
        const double ob2 = 0.09375 * xa;         // 3/32
        if (in_rc) {
            double s1, s2;
            smooth_part(p.alpha * r, p, s1, s2);
            c1 = ob1 - s1;
            c2 = ob2 - s2;
        } else {
            const double ar = p.a / r, ar3 = ar * ar * ar;
            c1 = ob1 - (0.75 * ar + 0.5 * ar3);
            c2 = ob2 - (0.75 * ar - 1.5 * ar3);
        }
    }
}

// b += c1 I + (c2 / r2) d d^T for an image d (r2 = |d|^2).
RPY_HD inline void add_coeffs(double dx, double dy, double dz, double r2, double c1, double c2,
                              double b[6])
{
    b[0] += c1;
    b[3] += c1;
    b[5] += c1;
    if (r2 > 0.0) {
        const double w = c2 / r2;
        b[0] += w * dx * dx;
        b[1] += w * dx * dy;
        b[2] += w * dx * dz;
        b[3] += w * dy * dy;
        b[4] += w * dy * dz;
        b[5] += w * dz * dz;
    }
}

RPY_HD inline void add_image(double dx, double dy, double dz, const PairConst &p,
                             double b[6])
{
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (!(r2 <= p.rc2) && !(r2 < p.a2x4)) return;
    double c1, c2;
    image_coeffs(r2, p, c1, c2);
    add_coeffs(dx, dy, dz, r2, c1, c2, b);
}

RPY_HD inline int image_lo(double d, const PairConst &p)
{
    return (int)ceil((-p.reach - d) * p.invL - 1e-12);
}
RPY_HD inline int image_hi(double d, const PairConst &p)
{
    return (int)floor((p.reach - d) * p.invL + 1e-12);
}

// Sum over all periodic images of one pair with wrapped separation d0
// (components in (-L, L)); for a bead with itself, the zero image is
// omitted and the self term added (eq. DF, first term and primed sum).
RPY_HD inline void pair_block(double d0x, double d0y, double d0z, bool self,
                              const PairConst &p, double b[6])
{
    for (int k = 0; k < 6; ++k) b[k] = 0.0;
    const int xl = image_lo(d0x, p), xh = image_hi(d0x, p);
    const int yl = image_lo(d0y, p), yh = image_hi(d0y, p);
    const int zl = image_lo(d0z, p), zh = image_hi(d0z, p);
    for (int nx = xl; nx <= xh; ++nx) {
        const double dx = d0x + nx * p.L;
        for (int ny = yl; ny <= yh; ++ny) {
            const double dy = d0y + ny * p.L;
            for (int nz = zl; nz <= zh; ++nz) {
                if (self && nx == 0 && ny == 0 && nz == 0) continue;
                add_image(dx, dy, d0z + nz * p.L, p, b);
            }
        }
    }
    if (self) {
        b[0] += p.self_coeff;
        b[3] += p.self_coeff;
        b[5] += p.self_coeff;
    }
}

PairConst make_pair_const(double L, double a, double alpha, double rc);

// ------------------------------------------------------- pair derivatives
// d/dx of the M1 coefficients (eq. M1 differentiated, x = alpha r), with the
// values: c1 = erfc(x) A + g B, c2 = erfc(x) A2 + g B2, g = e^{-x^2}/sqrt(pi),
// d erfc/dx = -2 g, dg/dx = -2 x g.
RPY_HD inline void m1_dcoeffs(double x, const PairConst &p, double &c1, double &c2, double &d1,
                              double &d2)
{
    const double x2 = x * x;
    const double e = erfc(x);
    const double g = exp(-x2) * p.inv_sqrtpi;
    const double ix = 1.0 / x, ix2 = ix * ix, ix3 = ix2 * ix, ix4 = ix2 * ix2;
    const double A = 0.75 * p.A1 * ix + 0.5 * p.A3 * ix3;
    const double Ap = -0.75 * p.A1 * ix2 - 1.5 * p.A3 * ix4;
    const double B = p.A1 * (3.0 * x2 - 4.5) + p.A3 * ((4.0 * x2 - 20.0) * x2 + 14.0 + ix2);
    const double Bp = 6.0 * p.A1 * x + p.A3 * ((16.0 * x2 - 40.0) * x - 2.0 * ix3);
    const double A2 = 0.75 * p.A1 * ix - 1.5 * p.A3 * ix3;
    const double A2p = -0.75 * p.A1 * ix2 + 4.5 * p.A3 * ix4;
    const double B2 = p.A1 * (1.5 - 3.0 * x2) + p.A3 * ((16.0 - 4.0 * x2) * x2 - 2.0 - 3.0 * ix2);
    const double B2p = -6.0 * p.A1 * x + p.A3 * ((32.0 - 16.0 * x2) * x + 6.0 * ix3);
    c1 = e * A + g * B;
    c2 = e * A2 + g * B2;
    d1 = -2.0 * g * A + e * Ap + g * (Bp - 2.0 * x * B);
    d2 = -2.0 * g * A2 + e * A2p + g * (B2p - 2.0 * x * B2);
}

// The smooth part S = Omega_A - M1 (see smooth_part) and its x-derivative:
// below XSER the derivative of the power series in x^2, else the closed form
// differentiated (d erf/dx = 2 g).
RPY_HD inline void smooth_dpart(double x, const PairConst &p, double &s1, double &s2, double &ds1,
                                double &ds2)
{
    const double x2 = x * x;
    if (x < XSER) {
        double u = p.s1[NSER - 1], v = p.s2[NSER - 1];
        double du = (NSER - 1) * p.s1[NSER - 1], dv = (NSER - 1) * p.s2[NSER - 1];
        for (int n = NSER - 2; n >= 1; --n) {
            u = u * x2 + p.s1[n];
            v = v * x2 + p.s2[n];
            du = du * x2 + n * p.s1[n];
            dv = dv * x2 + n * p.s2[n];
        }
        s1 = u * x2 + p.s1[0];
        s2 = v * x2 + p.s2[0];
        ds1 = 2.0 * x * du;
        ds2 = 2.0 * x * dv;
    } else {
        const double ef = erf(x);
        const double g = exp(-x2) * p.inv_sqrtpi;
        const double ix = 1.0 / x, ix2 = ix * ix, ix3 = ix2 * ix, ix4 = ix2 * ix2;
        const double P1 = 3.0 * x2 - 4.5, P1p = 6.0 * x;
        const double Q1 = (4.0 * x2 - 20.0) * x2 + 14.0 + ix2, Q1p = (16.0 * x2 - 40.0) * x - 2.0 * ix3;
        const double P2 = 1.5 - 3.0 * x2, P2p = -6.0 * x;
        const double Q2 = (16.0 - 4.0 * x2) * x2 - 2.0 - 3.0 * ix2,
                     Q2p = (32.0 - 16.0 * x2) * x + 6.0 * ix3;
        const double e1 = ef * ix, e1p = 2.0 * g * ix - ef * ix2;
        const double e3 = ef * ix3, e3p = 2.0 * g * ix3 - 3.0 * ef * ix4;
        s1 = p.A1 * (0.75 * e1 - P1 * g) + p.A3 * (0.5 * e3 - Q1 * g);
        s2 = p.A1 * (0.75 * e1 - P2 * g) + p.A3 * (-1.5 * e3 - Q2 * g);
        ds1 = p.A1 * (0.75 * e1p - (P1p - 2.0 * x * P1) * g) +
              p.A3 * (0.5 * e3p - (Q1p - 2.0 * x * Q1) * g);
        ds2 = p.A1 * (0.75 * e1p - (P2p - 2.0 * x * P2) * g) +
              p.A3 * (-1.5 * e3p - (Q2p - 2.0 * x * Q2) * g);
    }
}

// Gradient with respect to the image separation d of Ws : (c1 I + c2 dhat
// dhat) for one image (branches as add_image), Ws symmetric
// {xx, xy, xz, yy, yz, zz}:
//   grad = c1' dhat tr(Ws) + c2' dhat (dhat.Ws.dhat) + (c2/r)(2 Ws dhat - 2 dhat (dhat.Ws.dhat)),
// primes = d/dr.  The pair term is not differentiable at r = 0; nothing is
// added there.
RPY_HD inline void add_image_grad(double dx, double dy, double dz, const PairConst &p,
                                  const double Ws[6], double gr[3])
{
    const double r2 = dx * dx + dy * dy + dz * dz;
    const bool in_rc = r2 <= p.rc2;
    const bool ov = r2 < p.a2x4;
    if ((!in_rc && !ov) || r2 == 0.0) return;
    const double r = sqrt(r2);
    double c2, d1, d2;
    if (!ov) {
        double c1, e1, e2;
        m1_dcoeffs(p.alpha * r, p, c1, c2, e1, e2);
        d1 = p.alpha * e1;
        d2 = p.alpha * e2;
    } else if (in_rc) {
        double s1, s2, e1, e2;
        smooth_dpart(p.alpha * r, p, s1, s2, e1, e2);
        c2 = 0.09375 * r / p.a - s2;
        d1 = -0.28125 / p.a - p.alpha * e1;
        d2 = 0.09375 / p.a - p.alpha * e2;
    } else {
        const double ar = p.a / r, ar3 = ar * ar * ar;
        c2 = 0.09375 * r / p.a - (0.75 * ar - 1.5 * ar3);
        d1 = -0.28125 / p.a + (0.75 * ar + 1.5 * ar3) / r;
        d2 = 0.09375 / p.a + (0.75 * ar - 4.5 * ar3) / r;
    }
    const double ir = 1.0 / r;
    const double hx = dx * ir, hy = dy * ir, hz = dz * ir;
    const double tr = Ws[0] + Ws[3] + Ws[5];
    const double wx = Ws[0] * hx + Ws[1] * hy + Ws[2] * hz;
    const double wy = Ws[1] * hx + Ws[3] * hy + Ws[4] * hz;
    const double wz = Ws[2] * hx + Ws[4] * hy + Ws[5] * hz;
    const double hwh = hx * wx + hy * wy + hz * wz;
    const double a0 = d1 * tr + d2 * hwh - 2.0 * c2 * ir * hwh;
    const double b0 = 2.0 * c2 * ir;
    gr[0] += a0 * hx + b0 * wx;
    gr[1] += a0 * hy + b0 * wy;
    gr[2] += a0 * hz + b0 * wz;
}



// Sum over the periodic images of one pair of distinct beads with wrapped
// separation d0 of the gradient of Ws : D_pair(d) (add_image_grad).
RPY_HD inline void pair_grad(double d0x, double d0y, double d0z, const PairConst &p,
                             const double Ws[6], double gr[3])
{
    const int xl = image_lo(d0x, p), xh = image_hi(d0x, p);
    const int yl = image_lo(d0y, p), yh = image_hi(d0y, p);
    const int zl = image_lo(d0z, p), zh = image_hi(d0z, p);
    for (int nx = xl; nx <= xh; ++nx) {
        const double dx = d0x + nx * p.L;
        for (int ny = yl; ny <= yh; ++ny) {
            const double dy = d0y + ny * p.L;
            for (int nz = zl; nz <= zh; ++nz) add_image_grad(dx, dy, d0z + nz * p.L, p, Ws, gr);
        }
    }
}

// --------------------------------------------------------------- k-space
// Half-space wave-vector set: n with |n|^2 <= n2max and n > 0 in
// lexicographic (x, y, z) order; each carries weight 2 m(k) (the +-k pair)
// and khat.
struct KVec {
    int nx, ny, nz, pad;
};
struct KCoef {
    double w;          // 2 m(k)
    double hx, hy, hz; // khat
};

// ------------------------------------------------------------------ noise
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): round function
// (c0,c1,c2,c3) -> (hi(B c2) ^ c1 ^ k0, lo(B c2), hi(A c0) ^ c3 ^ k1, lo(A c0))
// with A = 0xD2511F53, B = 0xCD9E8D57, key bumped by (0x9E3779B9, 0xBB67AE85).
__device__ inline uint4 philox10(uint4 c, uint2 k)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
        k.x += 0x9E3779B9u;
        k.y += 0xBB67AE85u;
    }
    return c;
}

// ------------------------------------------------- adaptive Chebyshev order
// Device state of the adaptive order (eq. nint, then one more term until
// E_f < tol).  The host enqueues every product and trial an adaptive call may
// need up to its largest order; once a trial settles the order, `done` is set
// and the kernels of the later products and trials return at once, so no
// host synchronisation is needed.
struct AdaptState {
    int done;             // the order of the current call is settled
    int n_used;           // the settled order
    int n_start;          // first order tried by the current call
    int last_etol;        // the current call settled at its largest order with E_f >= tol
    long long etol;       // calls settled above the tolerance since the last status read
    long long calls;      // settled calls since the last order-statistics read
    long long sum_orders; // sum of their orders
    long long missed;     // those of them settled above the tolerance
    int max_order;        // largest of their orders
    int pad;
};

// -------------------------------------------------------------- context
struct Ctx {
    // problem
    int N, n3, nchains, bpc;
    double L, a, alpha, rc, kc;
    int n2max, nmax;   // |n|^2 cutoff and max |component|
    int nk;            // half-space wave vectors
    int lowp, max_rhs;
    int rhs_cap;       // stride of the per-RHS work buffers: max(max_rhs, 3)
    PairConst pc;
    // tiling
    int nbt;           // bead tiles per side
    int ntiles;        // stored tiles
    int n3pad;         // nbt * TS
    int nsfc;          // structure-factor bead chunks (SF_BEADS beads each)
    int lds_max = 48 * 1024;           // LDS bytes a workgroup may use on this device
    mutable unsigned symv_calls = 0;   // tile products launched (their parity sets the tile order)
    // Set by the profiler around one tile-product launch: that launch records
    // the pair itself (start and end of the kernel) and clears it.
    mutable hipEvent_t prof_ev0 = nullptr, prof_ev1 = nullptr;
    // device buffers
    double *rt = nullptr;        // wrapped positions [N][3] of the built D
    double *rt_ev = nullptr;     // wrapped positions for stand-alone force calls
    double *sfr = nullptr;       // fractional coordinates s = r/L - floor(r/L) [N][3]
    double2 *etab = nullptr;     // phases [N][3][nmax+1]
    KVec *kvec = nullptr;        // [nk]
    KCoef *kcoef = nullptr;      // [nk]
    int2 *tile_ij = nullptr;     // [ntiles]
    double *d64 = nullptr;       // [ntiles][TILE6], packed symmetric blocks
    float *p32 = nullptr;        // [ntiles][TILE6] packed planes, lowp FP32
    uint16_t *p16 = nullptr;     // [ntiles][TILE6] packed planes, lowp BF16
    double *part = nullptr;      // [nbt][rhs_cap][n3pad] tile-column partials
    // block products (5 to 16 vectors on the matrix cores, any tile precision)
    bool block = false;          // enabled: stored tiles and max_rhs >= BLOCK_MIN_RHS
    mutable int block_wgs[3] = {0, 0, 0};   // persistent grid of the tile kernel per precision
    int nchb;                    // bead chunks of the block structure factors
    int nk4;                     // nk rounded up to a multiple of 4
    void *xpk = nullptr;         // packed right-hand sides of the tile product (3 npad x 16 x 8 bytes)
    double *vpk = nullptr;       // the same vectors in FP64, [n3pad][16]
    void *bpart = nullptr;       // [nbt][n3pad][16] tile partials (FP64 for FP64 tiles, else FP32)
    double *tkm = nullptr;       // [nk4][6][16] 2 m(k) P_k (C_k, S_k), rows >= nk zero
    double *ypart = nullptr;     // [16][3N] summed FP64 tile partials of a block product
    double2 *eph = nullptr;      // [ceil(N/4)][nk16][4] e^{i k.r_mu} of the wrapped positions
    double *sfpart = nullptr;    // structure-factor partials (layouts in rpy_capi.hip)
    double *tk = nullptr;        // [nk][rhs_cap][6] 2 m(k) P_k (C_k, S_k)
    double *work = nullptr;      // vectors, see capi
    double *scal = nullptr;      // scalars: [0]=dmin [1]=dmax [2]=ya [3]=yb [8..]=coeffs
    double *red = nullptr;       // reduction outputs
    double *lanc = nullptr;      // [2 MAX_LANCZOS] Lanczos alpha, beta
    int cheb_keep = 0;           // Chebyshev vectors kept for the adaptive order
    double *vhist = nullptr;     // [cheb_keep][rhs_cap][3N]
    AdaptState *adapt = nullptr; // adaptive-order state
    double *tpart = nullptr;     // [rhs_cap][trial_chunks(N)][2] partial dot products of a trial
    // While set, every product kernel first reads *gate and returns at once
    // if it is non-zero (the products an adaptive call enqueues past the
    // order it may settle at).
    mutable const int *gate = nullptr;
    int *flags = nullptr;        // [0] nonfinite
    // low-memory (matrix-free) form: no stored tiles; the real-space part is
    // recomputed per product over a cell list of side >= max(r_c, 2a)
    bool lma = false;
    int nslot = 0;               // tile-column slots summed by the back-projection (1 for lma)
    int lma_nc = 0;              // cells per side
    int *lma_start = nullptr;    // [lma_nc^3 + 1] + cursor area [lma_nc^3]
    int *lma_beads = nullptr;    // [N] beads sorted by cell
    double *rt_sorted = nullptr; // [N][3] wrapped positions in cell order
    double *v_sorted = nullptr;  // [rhs_cap][N][3] product input in cell order
    // reverse mode (allocated when created with grad != 0)
    bool grad = false;
    double *wgrad = nullptr;     // [ntiles][TS*TS] W = sum_q x_q y_q^T + y_q x_q^T, stored tiles
    double *xy = nullptr;        // [cheb_keep][2][3N] adjoint pairs (x_q, y_q)
    double *gpart = nullptr;     // [nbt][n3pad] real-space gradient partials per tile column
    double *gk = nullptr;        // [3N] reciprocal-space gradient
    double *mur = nullptr;       // [3][3N] adjoint vectors mu_p (ring)
    // cell list for excluded volume
    int ncell;                   // cells per side (0: no cell list)
    int *cell_start = nullptr;   // [ncell^3 + 1]
    int *cell_beads = nullptr;   // [N]
    size_t work_elems = 0;
    double ev_rcut_built = 0.0;
};

// ------------------------------------------------------------ errors
// Parameter checks of rpy_create (RPY_OK or an error code; *n2max = the
// integer |n|^2 cutoff of the wave vectors), and the message rpy_strerror
// reports for the last RPY_EINVAL / RPY_ENOMEM / RPY_EHIP of this thread.
int validate_params(const rpy_params *p, int *n2max);
void set_error(const char *msg);
int hip_error(hipError_t e, const char *what);   // records and returns RPY_EHIP

// ------------------------------------------------------------ launchers
// build
void launch_wrap_tables(const Ctx &c, const double *pos, hipStream_t s);
// wrapped positions only (into `rt`), for forces of positions other than D's
void launch_wrap_positions(const Ctx &c, const double *pos, double *rt, hipStream_t s);
void launch_build_tiles(const Ctx &c, hipStream_t s);
void launch_dense_copy(const Ctx &c, double *out, hipStream_t s);
// products: the tile-product kernel also computes the structure-factor
// partials of its input; launch_sf_reduce turns them into tk; the final
// kernel adds the reciprocal back-projection to the tile partials and applies
// the epilogue of `mode`.
enum EpiMode { EPI_APPLY = 0, EPI_CHEB_FIRST = 1, EPI_CHEB_NEXT = 2, EPI_ADJ = 3 };
struct EpiArgs {
    int mode;
    int m;
    int p;                 // Chebyshev index of the vector being produced
    const double *vprev;   // V_{p-1} [m][3N]
    const double *vprev2;  // V_{p-2}
    double *vout;          // V_p, or D.v for EPI_APPLY
    double *acc;           // sum c_p V_p
    double *dv;            // optional: D.V_0 (EPI_CHEB_FIRST)
    const double *scal;    // device scalars (ya, yb, coeffs)
    double xs;             // EPI_ADJ: dv = xs * ya * vout
    int pack;              // block product: also write vout in the operand layouts of
    int pack_prec;         //   tiles of precision pack_prec (the next product's input)
    // Adaptive order (k_kspace_epi only): with trial_n > 0 the epilogue also
    // forms the trial of order trial_n from the vectors it has just written,
    // as k_trial_sum does -- dS = -c_0/2 V_0 + sum_{q < trial_n} c_q V_q
    // into ds, and per workgroup the partial sums of dS.dS and V_0.(D dW)
    // into tpart[j][workgroup][2] -- unless the order is settled or below
    // the call's first order; k_trial_check then reduces them.
    int trial_n;
    const AdaptState *adapt;
    const double *vhist;   // V_q at vhist + q ps
    size_t ps;
    const double *ddw;     // D.dW [m][3N]
    double *ds;            // dS [m][3N]
    double *tpart;
};
void launch_symv(const Ctx &c, int prec, const double *v, int j0, int mc, hipStream_t s);
// Block product D.V for 5 <= m <= 16 vectors (c.block): the tile product on
// the matrix cores from the packed planes of precision `prec` (FP64 or FP32
// partials), the FP64 matrix-core structure factors and their reduction to
// tkm (with the fixed-order sum of the partials), and the FP64 matrix-core
// back-projection fused with the epilogue `f`.
void launch_block_tiles(const Ctx &c, int prec, const double *v, int m, hipStream_t s,
                        bool packed = false);   // packed: the previous epilogue packed v
void launch_block_phases(const Ctx &c, hipStream_t s);   // eph from the current tables
void launch_block_sf(const Ctx &c, int m, int prec, hipStream_t s);
void launch_block_epi(const Ctx &c, const EpiArgs &f, hipStream_t s);
constexpr int BLOCK_MIN_RHS = 5;   // products with at least this many vectors use it
constexpr int BLOCK_RHS = 16;
void launch_sf_reduce(const Ctx &c, int m, hipStream_t s);
void launch_kspace_epi(const Ctx &c, const EpiArgs &f, hipStream_t s);
// Interval (explicit, or the paper's rule from du = D.U+), the scalars of Y
// and the coefficients of order n_cheb.  With adapt_floor >= 0 the order is
// the adaptive call's first one instead: adapt_floor if >= 2, else eq. nint
// on the interval, clamped to [2, adapt_max]; the adaptive state is reset.
void launch_cheb_coeffs(const Ctx &c, int n_cheb, int rule, double C, double dmin,
                        double dmax, const double *du, hipStream_t s, int adapt_floor = -1,
                        int adapt_max = 0);
// One trial order n of an adaptive call over m right-hand sides whose V_p are
// kept at c.vhist (stride ps per p) and D.V_0 at ddw: dS of order n into ds,
// E_f; settles the order when every E_f < tol or n = nmax (then e_f is
// written), else puts the coefficients of order n + 1 in place.
void launch_trial(const Ctx &c, int m, int n, int nmax, double tol, size_t ps,
                  const double *ddw, double *ds, double *e_f, hipStream_t s);
// The same decision when the back-projection epilogue of the product that
// completed order n formed the trial (EpiArgs::trial_n): only the check.
void launch_trial_check(const Ctx &c, int m, int n, int nmax, double tol, double *e_f,
                        hipStream_t s);
// Partial-sum chunks of a trial per right-hand side: the larger of the
// separate trial kernel's (256 entries each) and the epilogue's (one per
// workgroup), which sizes c.tpart.
int trial_chunks(int N);
void launch_sqrt_error(const Ctx &c, int m, const double *dw, const double *ddw,
                       const double *ds, double *e_f, hipStream_t s);
void launch_fill(double *p, double v, size_t n, hipStream_t s);
// Lanczos and the adaptive Chebyshev order
void launch_lanczos_init(int n, const double *r, double *q, hipStream_t s);
void launch_lanczos_step(int n, int j, const double *q, double *w, double *qprev, double *ab,
                         hipStream_t s);
void launch_cheb_resum(int n3, int m, int n_cheb, size_t pstride, const double *scal,
                       const double *vh, double *out, hipStream_t s);
void launch_copy(double *dst, const double *src, size_t n, hipStream_t s);
// reverse mode of u = D F + p(D) dW (rpy_grad.hip)
void launch_adj_init(const Ctx &c, int p, double xs, const double *g, double *mu, double *xq,
                     hipStream_t s);
void launch_add(double *out, const double *a, const double *b, size_t n, hipStream_t s);
void launch_grad_wtiles(const Ctx &c, int nq, hipStream_t s);
void launch_grad_real(const Ctx &c, hipStream_t s);
void launch_grad_sf(const Ctx &c, const double *v, int nv, hipStream_t s);
void launch_grad_kspace(const Ctx &c, const double *xy, int nq, int accumulate, hipStream_t s);
void launch_grad_sum(const Ctx &c, double *gpos, hipStream_t s);
// step
void launch_spring_forces(const Ctx &c, const double *pos, double *F, hipStream_t s);
void launch_cell_list(const Ctx &c, const double *rt, double rcut, hipStream_t s);
void launch_cell_list_into(int N, double L, int nc, const double *rt, int *start, int *beads,
                           hipStream_t s);
// low-memory form (rpy_lma.hip): cell list + positions in cell order; the
// matrix-free real-space product into part slot 0 and the structure-factor
// partials of the product's input
void launch_lma_build(const Ctx &c, hipStream_t s);
void launch_lma_real(const Ctx &c, const double *v, int m, hipStream_t s);
void launch_lma_sf(const Ctx &c, const double *v, int m, hipStream_t s);
void launch_ev_forces(const Ctx &c, const double *rt, double zstar, double dstar, double rcut,
                      double *F, hipStream_t s);
// g_pos += sum_mu J(d)(gF_nu - gF_mu): transpose of the excluded-volume Jacobian
void launch_ev_vjp(const Ctx &c, const double *rt, double zstar, double dstar, double rcut,
                   const double *gF, double *gpos, hipStream_t s);
void launch_noise(double *out, int64_t count, uint64_t seed, uint64_t step, double dt,
                  hipStream_t s);
void launch_philox(const uint32_t *ck, uint32_t *out, int64_t n, hipStream_t s);
void launch_cheb_first(const Ctx &c, const double *y, const double *v0, double *v1, double *acc,
                       double *dv, hipStream_t s);
void launch_euler(const Ctx &c, double *pos, double dt, const double *ud,
                  const double *ds, hipStream_t s);
void launch_observables(const Ctx &c, const double *pos, double *re2, double *rg2,
                        hipStream_t s);

}  // namespace rpy
