// rpy_capi.hip -- the C ABI declared in include/rpy.h: parameter validation,
// one-time allocation, wave-vector tables and the orchestration of every
// entry point on the caller's stream.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <vector>

#include "rpy_internal.h"

using namespace rpy;

struct Prof {
    int cap = 0;          // event pairs per kind (0: recording off)
    int alloc = 0;        // pairs created
    hipEvent_t *ev[RPY_PROF_KINDS] = {};
    int n[RPY_PROF_KINDS] = {};
};

struct rpy_ctx {
    Ctx c;
    Prof prof;
    double *F = nullptr;      // [3][3N]: forces, U+ (all ones), the step's dW
    double *Um = nullptr;     // [3N]: U- (alternating +1, -1 over the flattened index)
    double *Y = nullptr;      // [4][3N]: D.F, then D.U+, D.U-, D.dW as the step needs them
    double *dW = nullptr;     // [3N]
    double *dS = nullptr;     // [3N]
    double *Bv[2] = {nullptr, nullptr};  // [max_rhs][3N] Chebyshev vectors
    double *ddw = nullptr;    // [max_rhs][3N] D.dW
    double *acc = nullptr;    // [max_rhs][3N] scratch accumulator
    // the phase matrix c.eph is valid for wrap generation eph_gen
    uint64_t wrap_gen = 1, eph_gen = 0;
    // bd_step runs the forces and the noise on a second stream (default
    // priority) beside the tile build: fork after the wrap, join before the
    // drift product
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};

static thread_local char g_err[256];

static int hip_fail(hipError_t e, const char *what)
{
    snprintf(g_err, sizeof g_err, "%s: %s", what, hipGetErrorString(e));
    return RPY_EHIP;
}

#define HIP_TRY(x)                                  \
    do {                                            \
        hipError_t e_ = (x);                        \
        if (e_ != hipSuccess) return hip_fail(e_, #x); \
    } while (0)

static int check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, what);
    return RPY_OK;
}

namespace rpy {

// Series of the smooth part S = Omega_A - M1 in x^2 (x = alpha r), from
// erf(x)/x = (2/sqrt pi) sum (-1)^n x^{2n}/(n!(2n+1)) and
// e^{-x^2} = sum (-1)^n x^{2n}/n!:
//   f1_n = (-1)^n/n! [3/(2(2n+1)) + 9/2 + 3n]
//   g1_n = (-1)^n [1/(n+1)! - 1/((n+1)!(2n+3)) - (14 + 20n + 4n(n-1))/n!]
//   f2_n = (-1)^n/n! [3/(2(2n+1)) - 3/2 - 3n]
//   g2_n = (-1)^n [3/((n+1)!(2n+3)) - 3/(n+1)! + (2 + 16n + 4n(n-1))/n!]
// S1 = (A1 sum f1_n x^2n + A3 sum g1_n x^2n)/sqrt(pi), S2 likewise.
PairConst make_pair_const(double L, double a, double alpha, double rc)
{
    PairConst p;
    memset(&p, 0, sizeof p);
    p.L = L;
    p.invL = 1.0 / L;
    p.a = a;
    p.alpha = alpha;
    p.rc = rc;
    p.rc2 = rc * rc;
    p.reach = rc > 2.0 * a ? rc : 2.0 * a;
    p.a2x4 = 4.0 * a * a;
    p.inv_sqrtpi = 1.0 / sqrt(M_PI);
    p.A1 = a * alpha;
    p.A3 = p.A1 * p.A1 * p.A1;
    p.inv_A1sq = 1.0 / (p.A1 * p.A1);
    p.self_coeff = 1.0 - 6.0 * p.A1 * p.inv_sqrtpi + 40.0 * p.A3 * p.inv_sqrtpi / 3.0;
    double fact = 1.0;  // n!
    for (int n = 0; n < NSER; ++n) {
        if (n > 0) fact *= n;
        const double fact1 = fact * (n + 1);  // (n+1)!
        const double sg = (n & 1) ? -1.0 : 1.0;
        const double f1 = sg / fact * (3.0 / (2.0 * (2 * n + 1)) + 4.5 + 3.0 * n);
        const double g1 = sg * (1.0 / fact1 - 1.0 / (fact1 * (2 * n + 3))
                                - (14.0 + 20.0 * n + 4.0 * n * (n - 1)) / fact);
        const double f2 = sg / fact * (3.0 / (2.0 * (2 * n + 1)) - 1.5 - 3.0 * n);
        const double g2 = sg * (3.0 / (fact1 * (2 * n + 3)) - 3.0 / fact1
                                + (2.0 + 16.0 * n + 4.0 * n * (n - 1)) / fact);
        p.s1[n] = (p.A1 * f1 + p.A3 * g1) * p.inv_sqrtpi;
        p.s2[n] = (p.A1 * f2 + p.A3 * g2) * p.inv_sqrtpi;
    }
    return p;
}

}  // namespace rpy

static int validate(const rpy_params *p, int *n2max_out)
{
    if (!p) return RPY_EINVAL;
    if (p->n_beads <= 0 || !(p->box_l > 0) || !(p->a > 0) || !(p->alpha > 0) || !(p->r_c > 0) ||
        !(p->k_c > 0) || !isfinite(p->box_l) || !isfinite(p->a) || !isfinite(p->alpha) ||
        !isfinite(p->r_c) || !isfinite(p->k_c)) {
        snprintf(g_err, sizeof g_err, "non-positive or non-finite size or Ewald parameter");
        return RPY_EINVAL;
    }
    if (p->n_chains <= 0 || p->beads_per_chain <= 0 ||
        (int64_t)p->n_chains * p->beads_per_chain != p->n_beads) {
        snprintf(g_err, sizeof g_err, "n_chains * beads_per_chain must equal n_beads");
        return RPY_EINVAL;
    }
    if (p->max_rhs < 1 || p->max_rhs > MAX_RHS) {
        snprintf(g_err, sizeof g_err, "max_rhs must be in 1..%d", MAX_RHS);
        return RPY_EINVAL;
    }
    if (p->lma != 0 && p->lma != 1) {
        snprintf(g_err, sizeof g_err, "lma must be 0 or 1");
        return RPY_EINVAL;
    }
    if (p->lma && p->grad) {
        snprintf(g_err, sizeof g_err, "grad needs the stored form (lma = 0)");
        return RPY_EINVAL;
    }
    if (p->lma) {
        const double reach = p->r_c > 2.0 * p->a ? p->r_c : 2.0 * p->a;
        if (!(3.0 * reach <= p->box_l)) {
            snprintf(g_err, sizeof g_err, "lma needs max(r_c, 2a) <= L/3 (3 cells per side)");
            return RPY_EINVAL;
        }
    }
    if (p->grad != 0 && p->grad != 1) {
        snprintf(g_err, sizeof g_err, "grad must be 0 or 1");
        return RPY_EINVAL;
    }
    if (p->grad && p->cheb_keep < 2) {
        snprintf(g_err, sizeof g_err, "grad needs cheb_keep >= 2 (the Chebyshev terms kept)");
        return RPY_EINVAL;
    }
    if (p->cheb_keep < 0 || p->cheb_keep > MAX_NCHEB) {
        snprintf(g_err, sizeof g_err, "cheb_keep must be in 0..%d", MAX_NCHEB);
        return RPY_EINVAL;
    }
    if (p->lowp != RPY_PREC_F64 && p->lowp != RPY_PREC_F32 && p->lowp != RPY_PREC_BF16) {
        snprintf(g_err, sizeof g_err, "unknown lowp");
        return RPY_EINVAL;
    }
    if (!(4.0 * p->a < p->box_l)) {
        snprintf(g_err, sizeof g_err, "box too small: need 4a < L");
        return RPY_EGEOM;
    }
    const double q = p->k_c * p->box_l / (2.0 * M_PI);
    const double n2 = floor(q * q);
    if (n2 < 1.0 || n2 > 255.0) {
        snprintf(g_err, sizeof g_err, "wave-vector cutoff gives |n|^2 <= %.0f (need 1..255)", n2);
        return RPY_EINVAL;
    }
    // real-space images per axis must stay bounded
    if (p->r_c > 64.0 * p->box_l) {
        snprintf(g_err, sizeof g_err, "r_c > 64 L");
        return RPY_EINVAL;
    }
    *n2max_out = (int)n2;
    return RPY_OK;
}

namespace rpy {
int validate_params(const rpy_params *p, int *n2max) { return validate(p, n2max); }
void set_error(const char *msg) { snprintf(g_err, sizeof g_err, "%s", msg); }
int hip_error(hipError_t e, const char *what) { return hip_fail(e, what); }
}  // namespace rpy

// Structure-factor partials: [nsfc][6 rhs_cap][nk] for the vector-unit
// product, [nk/16 blocks][nchb][6 x 16][16] for the block product.
static size_t sfpart_elems(const Ctx &c)
{
    const size_t a = (size_t)c.nsfc * 6 * c.rhs_cap * c.nk;
    const size_t b = c.block ? (size_t)((c.nk + 15) / 16) * c.nchb * 6 * BLOCK_RHS * 16 : 0;
    return a > b ? a : b;
}

template <typename T> static int dalloc(T **p, size_t n)
{
    if (n == 0) n = 1;
    hipError_t e = hipMalloc((void **)p, n * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        snprintf(g_err, sizeof g_err, "hipMalloc(%zu bytes): %s", n * sizeof(T),
                 hipGetErrorString(e));
        return RPY_ENOMEM;
    }
    return RPY_OK;
}

extern "C" void rpy_destroy(rpy_ctx *x)
{
    if (!x) return;
    (void)hipDeviceSynchronize();
    Ctx &c = x->c;
    void *bufs[] = {c.rt, c.rt_ev, c.eph, c.etab, c.kvec, c.kcoef, c.tile_ij, c.d64,
                    c.p32, c.p16, c.part, c.xpk, c.ypart,
                    c.vpk, c.bpart, c.tkm,
                    c.sfpart, c.tk, c.sfr, c.work, c.scal, c.red, c.flags, c.cell_start, c.lanc,
                    c.adapt, c.tpart,
                    c.vhist, c.wgrad, c.xy, c.gpart, c.gk, c.mur,
                    c.lma_start, c.lma_beads, c.rt_sorted, c.v_sorted,
                    c.cell_beads};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    if (x->fork) (void)hipEventDestroy(x->fork);
    if (x->join) (void)hipEventDestroy(x->join);
    if (x->side) (void)hipStreamDestroy(x->side);
    for (int k = 0; k < RPY_PROF_KINDS; ++k) {
        for (int i = 0; i < 2 * x->prof.alloc; ++i) (void)hipEventDestroy(x->prof.ev[k][i]);
        delete[] x->prof.ev[k];
    }
    delete x;
}

extern "C" int rpy_create(rpy_ctx **out, const rpy_params *p)
{
    if (!out) return RPY_EINVAL;
    *out = nullptr;
    int n2max = 0;
    int rc = validate(p, &n2max);
    if (rc) return rc;
    rpy_ctx *x = new (std::nothrow) rpy_ctx();
    if (!x) return RPY_ENOMEM;
    Ctx &c = x->c;
    c.N = p->n_beads;
    c.n3 = 3 * c.N;
    c.nchains = p->n_chains;
    c.bpc = p->beads_per_chain;
    c.L = p->box_l;
    c.a = p->a;
    c.alpha = p->alpha;
    c.rc = p->r_c;
    c.kc = p->k_c;
    c.n2max = n2max;
    c.nmax = (int)floor(sqrt((double)n2max));
    while ((c.nmax + 1) * (c.nmax + 1) <= n2max) ++c.nmax;
    while (c.nmax * c.nmax > n2max) --c.nmax;
    c.lowp = p->lowp;
    c.max_rhs = p->max_rhs;
    c.cheb_keep = p->cheb_keep;
    c.grad = p->grad != 0;
    c.lma = p->lma != 0;
    c.rhs_cap = c.max_rhs > 4 ? c.max_rhs : 4;   // bd_step's product of [F, U+, U-, dW]
    c.block = !c.lma && c.max_rhs >= BLOCK_MIN_RHS;
    if (c.block) c.rhs_cap = BLOCK_RHS;  // block kernels write all 16 columns
    {
        int dev = 0, lds = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
            lds > 0)
            c.lds_max = lds;
    }
    c.pc = make_pair_const(c.L, c.a, c.alpha, c.rc);
    c.nbt = (c.N + TB - 1) / TB;
    c.ntiles = c.nbt * (c.nbt + 1) / 2;
    c.n3pad = c.nbt * TS;
    c.nsfc = (c.N + SF_BEADS - 1) / SF_BEADS;
    c.nslot = c.nbt;
    if (c.lma) {   // no stored tiles: one partial slot, cells of side >= max(r_c, 2a)
        c.nslot = 1;
        c.lowp = RPY_PREC_F64;
        const int nc = (int)floor(c.L / c.pc.reach);
        c.lma_nc = nc > 128 ? 128 : nc;
    }

    // half-space wave vectors, lexicographically positive
    std::vector<KVec> kv;
    std::vector<KCoef> kc;
    const double vol = c.L * c.L * c.L;
    for (int nx = 0; nx <= c.nmax; ++nx)
        for (int ny = -c.nmax; ny <= c.nmax; ++ny)
            for (int nz = -c.nmax; nz <= c.nmax; ++nz) {
                const int n2 = nx * nx + ny * ny + nz * nz;
                if (n2 == 0 || n2 > n2max) continue;
                if (nx == 0 && (ny < 0 || (ny == 0 && nz < 0))) continue;
                const double kx = 2.0 * M_PI * nx / c.L, ky = 2.0 * M_PI * ny / c.L,
                             kz = 2.0 * M_PI * nz / c.L;
                const double k2 = kx * kx + ky * ky + kz * kz, k = sqrt(k2);
                const double al2 = c.alpha * c.alpha;
                const double mk = (c.a - c.a * c.a * c.a * k2 / 3.0) *
                                  (1.0 + k2 / (4.0 * al2) + k2 * k2 / (8.0 * al2 * al2)) *
                                  (6.0 * M_PI / (k2 * vol)) * exp(-k2 / (4.0 * al2));
                kv.push_back(KVec{nx, ny, nz, 0});
                kc.push_back(KCoef{2.0 * mk, kx / k, ky / k, kz / k});
            }
    c.nk = (int)kv.size();
    c.nk4 = (c.nk + 3) / 4 * 4;
    c.nchb = c.nsfc < 16 ? c.nsfc : 16;

    std::vector<int2> tij;
    for (int I = 0; I < c.nbt; ++I)
        for (int J = I; J < c.nbt; ++J) tij.push_back(make_int2(I, J));

    const size_t te = c.lma ? 0 : (size_t)c.ntiles * TILE_ELEMS;   // row-major W tiles (grad)
    const size_t te6 = c.lma ? 0 : (size_t)c.ntiles * TILE6;
    const size_t lcells = c.lma ? (size_t)c.lma_nc * c.lma_nc * c.lma_nc : 0;
    const size_t nv = (size_t)c.n3;
    const size_t mv = (size_t)c.rhs_cap * nv;
    c.work_elems = 3 * nv + nv + 4 * nv + nv + nv + 2 * mv + mv + mv;
    const int ncell_cap = 64;
    const size_t ncells_cap = (size_t)ncell_cap * ncell_cap * ncell_cap;
    if ((rc = dalloc(&c.rt, nv)) || (rc = dalloc(&c.rt_ev, nv)) || (rc = dalloc(&c.etab, nv * (c.nmax + 1))) ||
        (rc = dalloc(&c.kvec, kv.size())) || (rc = dalloc(&c.kcoef, kc.size())) ||
        (rc = dalloc(&c.tile_ij, tij.size())) || (!c.lma && (rc = dalloc(&c.d64, te6))) ||
        (c.lma && ((rc = dalloc(&c.lma_start, 2 * lcells + 1)) ||
                   (rc = dalloc(&c.lma_beads, (size_t)c.N)) ||
                   (rc = dalloc(&c.rt_sorted, nv)) ||
                   (rc = dalloc(&c.v_sorted, (size_t)c.rhs_cap * nv)))) ||
        (c.lowp == RPY_PREC_F32 && (rc = dalloc(&c.p32, te6))) ||
        (c.lowp == RPY_PREC_BF16 && (rc = dalloc(&c.p16, te6))) ||
        (rc = dalloc(&c.part, (size_t)c.nslot * c.rhs_cap * c.n3pad)) ||
        (c.block && ((rc = dalloc(reinterpret_cast<double **>(&c.xpk),
                                  (size_t)c.n3pad * BLOCK_RHS)) ||
                     (rc = dalloc(&c.vpk, (size_t)c.n3pad * BLOCK_RHS)) ||
                     (rc = dalloc(reinterpret_cast<double **>(&c.bpart),
                                  (size_t)c.nbt * BLOCK_RHS * c.n3pad)) ||
                     (rc = dalloc(&c.tkm, (size_t)c.nk4 * 6 * BLOCK_RHS)) ||
                     (rc = dalloc(&c.ypart, (size_t)BLOCK_RHS * c.n3)) ||
                     (rc = dalloc(&c.eph, (size_t)(c.N + 3) / 4 * ((c.nk + 15) / 16 * 16) * 4)))) ||
        (rc = dalloc(&c.sfpart, sfpart_elems(c))) ||
        (rc = dalloc(&c.tk, (size_t)6 * c.rhs_cap * c.nk)) ||
        (rc = dalloc(&c.sfr, nv)) ||
        (rc = dalloc(&c.work, c.work_elems)) || (rc = dalloc(&c.scal, 8 + MAX_NCHEB)) ||
        (rc = dalloc(&c.red, 64)) || (rc = dalloc(&c.flags, 4)) ||
        (rc = dalloc(&c.lanc, 2 * MAX_LANCZOS)) ||
        (rc = dalloc(&c.adapt, 1)) ||
        (rc = dalloc(&c.tpart, (size_t)c.rhs_cap * trial_chunks(c.N) * 2)) ||
        (c.cheb_keep > 0 && (rc = dalloc(&c.vhist, (size_t)c.cheb_keep * c.rhs_cap * nv))) ||
        (c.grad && ((rc = dalloc(&c.wgrad, te)) ||
                    (rc = dalloc(&c.xy, (size_t)c.cheb_keep * 2 * nv)) ||
                    (rc = dalloc(&c.gpart, (size_t)c.nbt * c.n3pad)) ||
                    (rc = dalloc(&c.gk, nv)) || (rc = dalloc(&c.mur, 3 * nv)))) ||
        (rc = dalloc(&c.cell_start, 2 * ncells_cap + 1)) || (rc = dalloc(&c.cell_beads, nv))) {
        rpy_destroy(x);
        return rc;
    }
    double *w = c.work;
    x->F = w; w += 3 * nv;
    x->Um = w; w += nv;
    x->Y = w; w += 4 * nv;
    x->dW = w; w += nv;
    x->dS = w; w += nv;
    x->Bv[0] = w; w += mv;
    x->Bv[1] = w; w += mv;
    x->ddw = w; w += mv;
    x->acc = w; w += mv;
    std::vector<double> um(nv);
    for (size_t i = 0; i < nv; ++i) um[i] = (i & 1) ? -1.0 : 1.0;
    hipError_t e;
    if ((e = hipMemcpy(c.kvec, kv.data(), kv.size() * sizeof(KVec), hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(x->Um, um.data(), nv * sizeof(double), hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(c.kcoef, kc.data(), kc.size() * sizeof(KCoef), hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(c.tile_ij, tij.data(), tij.size() * sizeof(int2), hipMemcpyHostToDevice)) ||
        (e = hipMemset(c.flags, 0, 4 * sizeof(int))) ||
        (e = hipMemset(c.adapt, 0, sizeof(AdaptState))) ||
        (te6 && (e = hipMemset(c.d64, 0, te6 * sizeof(double)))) ||
        (c.block && (e = hipMemset(c.tkm, 0, (size_t)c.nk4 * 6 * BLOCK_RHS * sizeof(double))))) {
        rc = hip_fail(e, "rpy_create upload");
        rpy_destroy(x);
        return rc;
    }
    if ((e = hipStreamCreateWithFlags(&x->side, hipStreamNonBlocking)) ||
        (e = hipEventCreateWithFlags(&x->fork, hipEventDisableTiming)) ||
        (e = hipEventCreateWithFlags(&x->join, hipEventDisableTiming))) {
        rc = hip_fail(e, "rpy_create stream");
        rpy_destroy(x);
        return rc;
    }
    launch_fill(x->F + nv, 1.0, nv, 0);   // U+ = (1, 1, ..., 1)
    if ((e = hipDeviceSynchronize()) != hipSuccess) {
        rc = hip_fail(e, "rpy_create sync");
        rpy_destroy(x);
        return rc;
    }
    *out = x;
    return RPY_OK;
}

static inline hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Event pair around one launch of kind k (no-op when recording is off).
struct ProfScope {
    rpy_ctx *x;
    int k;
    hipStream_t s;
    bool on;
    ProfScope(rpy_ctx *x_, int k_, hipStream_t s_) : x(x_), k(k_), s(s_)
    {
        // products an adaptive call enqueues past its first trial run under
        // the gate and may return at once: they are not recorded
        on = x->prof.cap > 0 && x->prof.n[k] < x->prof.cap && !x->c.gate;
        if (!on) return;
        hipEvent_t *e = &x->prof.ev[k][2 * x->prof.n[k]];
        (void)hipEventRecord(e[0], s);
        if (k == RPY_PROF_SYMV || k == RPY_PROF_SYMV_MULTI) {
            // a packed-tile launch in this scope takes the pair over and
            // records it from its own dispatch (kernel time only)
            x->c.prof_ev0 = e[0];
            x->c.prof_ev1 = e[1];
        }
    }
    ~ProfScope()
    {
        if (!on) return;
        const bool taken = (k == RPY_PROF_SYMV || k == RPY_PROF_SYMV_MULTI) && !x->c.prof_ev0;
        x->c.prof_ev0 = x->c.prof_ev1 = nullptr;
        if (!taken) (void)hipEventRecord(x->prof.ev[k][2 * x->prof.n[k] + 1], s);
        ++x->prof.n[k];
    }
};

extern "C" int rpy_ewald_build(rpy_ctx *x, const double *pos, void *stream)
{
    if (!x || !pos) return RPY_EINVAL;
    launch_wrap_tables(x->c, pos, S(stream));
    ++x->wrap_gen;
    {
        ProfScope ps(x, RPY_PROF_BUILD, S(stream));
        launch_build_tiles(x->c, S(stream));
    }
    return check_launch("rpy_ewald_build");
}

static bool prec_ok(const Ctx &c, int prec)
{
    return prec == RPY_PREC_F64 || (prec == RPY_PREC_F32 && c.lowp == RPY_PREC_F32) ||
           (prec == RPY_PREC_BF16 && c.lowp == RPY_PREC_BF16);
}

// One product of the full periodic D with the m vectors v; `f` selects the
// epilogue.  Two kernels per group of up to 4 vectors: the tile product
// (whose structure-factor workgroups also write T_k of v), then the
// reciprocal back-projection + epilogue.  With 5..16 vectors the block path
// runs instead: matrix-core tile product, FP64 matrix-core structure factors
// and back-projection.  The low-memory form: the matrix-free real-space
// product, structure-factor partials, their reduction, the back-projection.
// prepacked: v is the output of the previous product of the same series,
// whose block epilogue (f.pack) already wrote it in the packed layouts.
static void product(rpy_ctx *x, const double *v, int m, int prec, const EpiArgs &f,
                    hipStream_t s, bool prepacked = false)
{
    const Ctx &c = x->c;
    if (c.lma) {   // matrix-free real space + structure factors of v
        {
            ProfScope ps(x, RPY_PROF_SYMV, s);
            launch_lma_real(c, v, m, s);
        }
        {
            ProfScope ps(x, RPY_PROF_KSPACE, s);
            launch_lma_sf(c, v, m, s);
            launch_sf_reduce(c, m, s);
        }
        ProfScope ps(x, RPY_PROF_EPI, s);
        launch_kspace_epi(c, f, s);
        return;
    }
    if (c.block && m >= BLOCK_MIN_RHS) {
        {
            ProfScope ps(x, RPY_PROF_SYMV, s);
            launch_block_tiles(c, prec, v, m, s, prepacked);
        }
        {
            ProfScope ps(x, RPY_PROF_KSPACE, s);
            if (x->eph_gen != x->wrap_gen) {   // positions changed since the last phases
                launch_block_phases(c, s);
                x->eph_gen = x->wrap_gen;
            }
            launch_block_sf(c, m, prec, s);
        }
        ProfScope ps(x, RPY_PROF_EPI, s);
        launch_block_epi(c, f, s);
        return;
    }
    // the tile-product launches also write T_k of their vectors
    for (int j0 = 0; j0 < m;) {
        const int r = m - j0;
        const int mc = r >= 4 ? 4 : r;
        ProfScope ps(x, mc == 1 ? RPY_PROF_SYMV : RPY_PROF_SYMV_MULTI, s);
        launch_symv(c, prec, v, j0, mc, s);
        j0 += mc;
    }
    ProfScope ps(x, RPY_PROF_EPI, s);
    launch_kspace_epi(c, f, s);
}

extern "C" int rpy_apply(rpy_ctx *x, const double *v, double *out, int m, int prec,
                         void *stream)
{
    if (!x || !v || !out || m < 1 || m > x->c.max_rhs || !prec_ok(x->c, prec)) return RPY_EINVAL;
    EpiArgs f{};
    f.mode = EPI_APPLY;
    f.m = m;
    f.vout = out;
    product(x, v, m, prec, f, S(stream));
    return check_launch("rpy_apply");
}

// Chebyshev recurrence with coefficients already in c.scal.
// Products p = first .. n_cheb - 1 of the recurrence (first = 2 when V_1,
// acc and D.dW are already in Bv[1], out and ddw).
static void cheb_run(rpy_ctx *x, const double *dw, double *out, int m, int n_cheb, int prec,
                     hipStream_t s, int first = 1)
{
    const Ctx &c = x->c;
    for (int p = first; p < n_cheb; ++p) {
        EpiArgs f{};
        f.m = m;
        f.p = p;
        f.scal = c.scal;
        f.acc = out;
        if (p == 1) {
            f.mode = EPI_CHEB_FIRST;
            f.vprev = dw;
            f.vout = x->Bv[1];
            f.dv = x->ddw;
        } else {
            f.mode = EPI_CHEB_NEXT;
            f.vprev = x->Bv[(p - 1) % 2];
            f.vprev2 = p == 2 ? dw : x->Bv[p % 2];
            f.vout = x->Bv[p % 2];
        }
        f.pack = p + 1 < n_cheb;   // V_p is the next product's input
        f.pack_prec = prec;
        product(x, f.vprev, m, prec, f, s, p > first);
    }
}

// First order of an adaptive call as the device computes it from the
// interval (eq. nint, rounded half away from zero) or the caller's start.
static int adapt_first(int floor_n, double d_min, double d_max, int nmax)
{
    int k = floor_n;
    if (floor_n < 2) {
        const double r = round(sqrt(d_max / d_min)) + 1.0;
        k = r < (double)nmax ? (int)r : nmax;
    }
    return k < 2 ? 2 : (k > nmax ? nmax : k);
}

// The adaptive order (eq. nint, then one more term at a time until E_f < tol
// for every right-hand side, section "Decomposition of the diffusion
// tensor").  On entry V_0 is in the history (c.vhist, stride ps per term)
// and launch_cheb_coeffs has reset the adaptive state and written the
// coefficients of the first order; with first = 2 V_1 and D.V_0 are in place
// as well.  Every product up to the largest order nmax is enqueued, each
// followed by a trial of the order it completes; the products after the first
// trial run under the gate, so that the kernels of everything past the
// settled order return at once.  host_first is the first order the device
// can start from (no trial is enqueued below it).  dS of the settled order
// ends in out, its E_f in e_f.  Where the product ends in k_kspace_epi (tile
// and matrix-free products; not the block product), that epilogue forms the
// trial of the order it completes, so that only the check is a launch of
// its own.
static void cheb_adapt_run(rpy_ctx *x, int m, int prec, int first, int host_first, int nmax,
                           double tol, double *out, double *e_f, hipStream_t s)
{
    Ctx &c = x->c;
    const size_t ps = (size_t)c.rhs_cap * c.n3;
    double *vh = c.vhist;
    const int *done = &c.adapt->done;
    auto trial = [&](int n, bool fused) {
        if (n < host_first) return;
        if (fused) launch_trial_check(c, m, n, nmax, tol, e_f, s);
        else launch_trial(c, m, n, nmax, tol, ps, x->ddw, out, e_f, s);
    };
    const bool fuse = !(c.block && m >= BLOCK_MIN_RHS);
    if (first == 2) trial(2, false);
    for (int p = first; p < nmax; ++p) {
        EpiArgs f{};
        f.m = m;
        f.p = p;
        f.scal = c.scal;
        f.acc = x->acc;   // the fixed-order running sum: not used by the trials
        f.vout = vh + p * ps;
        f.vprev = vh + (p - 1) * ps;
        if (p == 1) {
            f.mode = EPI_CHEB_FIRST;
            f.dv = x->ddw;
        } else {
            f.mode = EPI_CHEB_NEXT;
            f.vprev2 = vh + (p - 2) * ps;
        }
        f.pack = p + 1 < nmax;   // V_p is the next product's input
        f.pack_prec = prec;
        const bool fused = fuse && p + 1 >= host_first;
        if (fused) {
            f.trial_n = p + 1;
            f.adapt = c.adapt;
            f.vhist = vh;
            f.ps = ps;
            f.ddw = x->ddw;
            f.ds = out;
            f.tpart = c.tpart;
        }
        c.gate = p >= host_first ? done : nullptr;   // a trial may have settled the order
        product(x, f.vprev, m, prec, f, s, p > first);
        c.gate = nullptr;
        trial(p + 1, fused);
    }
}

// Reads the adaptive state after the stream has drained.
static int adapt_result(rpy_ctx *x, int *n_used, hipStream_t s)
{
    AdaptState st;
    HIP_TRY(hipMemcpyAsync(&st, x->c.adapt, sizeof st, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (n_used) *n_used = st.n_used;
    return st.last_etol ? RPY_ETOL : RPY_OK;
}

extern "C" int chebyshev_sqrt_apply(rpy_ctx *x, const double *dw, double *out, int m,
                                    int n_cheb, double d_min, double d_max, double tol, int prec,
                                    int *n_used, double *e_f, void *stream)
{
    if (!x || !dw || !out || m < 1 || m > x->c.max_rhs || n_cheb < 2 || n_cheb > MAX_NCHEB ||
        !(d_min > 0) || !(d_max > d_min) || !isfinite(d_max) || !prec_ok(x->c, prec) ||
        !(tol == tol) || tol == INFINITY)
        return RPY_EINVAL;
    hipStream_t s = S(stream);
    Ctx &c = x->c;
    if (tol > 0) {
        if (n_cheb > c.cheb_keep) {
            snprintf(g_err, sizeof g_err, "the adaptive order needs cheb_keep >= n_cheb");
            return RPY_EINVAL;
        }
        launch_copy(c.vhist, dw, (size_t)m * c.n3, s);   // V_0
        launch_cheb_coeffs(c, 0, RPY_BOUNDS_EXPLICIT, 0.0, d_min, d_max, nullptr, s, 0, n_cheb);
        cheb_adapt_run(x, m, prec, 1, adapt_first(0, d_min, d_max, n_cheb), n_cheb, tol, out,
                       e_f ? e_f : c.red, s);
        int rc = check_launch("chebyshev_sqrt_apply");
        if (rc || !n_used) return rc;
        return adapt_result(x, n_used, s);
    }
    launch_cheb_coeffs(c, n_cheb, RPY_BOUNDS_EXPLICIT, 0.0, d_min, d_max, nullptr, s);
    cheb_run(x, dw, out, m, n_cheb, prec, s);
    if (e_f) launch_sqrt_error(c, m, dw, x->ddw, out, e_f, s);
    if (n_used) *n_used = n_cheb;
    return check_launch("chebyshev_sqrt_apply");
}

// Number of eigenvalues of the symmetric tridiagonal (a, b) below x
// (Sturm sequence of the LDL^T pivots).
static int sturm_below(const double *a, const double *b, int k, double x)
{
    int cnt = 0;
    double q = 1.0;
    for (int i = 0; i < k; ++i) {
        const double off = i > 0 ? b[i - 1] * b[i - 1] / q : 0.0;
        q = a[i] - x - off;
        if (q == 0.0) q = -1e-300;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

// Eigenvalue number idx (0 = smallest) of the tridiagonal by bisection on
// the Gershgorin interval.
static double tridiag_eig(const double *a, const double *b, int k, int idx)
{
    double lo = a[0], hi = a[0];
    for (int i = 0; i < k; ++i) {
        const double r = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i + 1 < k ? fabs(b[i]) : 0.0);
        lo = fmin(lo, a[i] - r);
        hi = fmax(hi, a[i] + r);
    }
    for (int it = 0; it < 200 && hi - lo > 1e-15 * fmax(fabs(lo), fabs(hi)); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (sturm_below(a, b, k, mid) > idx) hi = mid;
        else lo = mid;
    }
    return 0.5 * (lo + hi);
}

// Solve (T - x I) y = r for the symmetric tridiagonal T = (a, b) by
// Gaussian elimination with partial pivoting (LAPACK's gtsv scheme).
static void tridiag_solve(const double *a, const double *b, int k, double x,
                          std::vector<double> &r)
{
    std::vector<double> dl(k), d(k), du(k), du2(k, 0.0);
    for (int i = 0; i < k; ++i) {
        d[i] = a[i] - x;
        du[i] = i + 1 < k ? b[i] : 0.0;
        dl[i] = i + 1 < k ? b[i] : 0.0;   // sub-diagonal entry below row i
    }
    for (int i = 0; i + 1 < k; ++i) {
        if (fabs(d[i]) >= fabs(dl[i])) {   // no row interchange
            const double f = d[i] != 0.0 ? dl[i] / d[i] : 0.0;
            d[i + 1] -= f * du[i];
            r[i + 1] -= f * r[i];
            dl[i] = 0.0;
        } else {                           // interchange rows i and i + 1
            const double f = d[i] / dl[i];
            d[i] = dl[i];
            const double t = d[i + 1];
            d[i + 1] = du[i] - f * t;
            if (i + 2 < k) {
                du2[i] = du[i + 1];
                du[i + 1] = -f * du2[i];
            }
            du[i] = t;
            const double rt = r[i];
            r[i] = r[i + 1];
            r[i + 1] = rt - f * r[i + 1];
        }
    }
    for (int i = k - 1; i >= 0; --i) {
        double v = r[i];
        if (i + 1 < k) v -= du[i] * r[i + 1];
        if (i + 2 < k) v -= du2[i] * r[i + 2];
        const double piv = d[i] != 0.0 ? d[i] : 1e-300;
        r[i] = v / piv;
    }
}

// |last component| of the unit eigenvector of the tridiagonal for the
// eigenvalue theta, by three steps of inverse iteration from a constant
// vector (the shift is moved off theta by a few ulps).
static double tridiag_last(const double *a, const double *b, int k, double th)
{
    const double x = th + 8.0 * 2.22e-16 * fmax(fabs(th), 1e-300);
    std::vector<double> r(k, 1.0);
    for (int it = 0; it < 3; ++it) {
        tridiag_solve(a, b, k, x, r);
        double n = 0.0;
        for (double v : r) n += v * v;
        n = sqrt(n);
        if (!(n > 0) || !isfinite(n)) return 1.0;   // no information: widest residual
        for (double &v : r) v /= n;
    }
    return fabs(r[k - 1]);
}

extern "C" int rpy_lanczos_bounds(rpy_ctx *x, int n_iter, uint64_t seed, const double *start,
                                  double margin, double *d_min, double *d_max, double *alpha,
                                  double *beta, void *stream)
{
    if (!x || !d_min || !d_max || n_iter < 2 || n_iter > MAX_LANCZOS || !(margin >= 0))
        return RPY_EINVAL;
    hipStream_t s = S(stream);
    const Ctx &c = x->c;
    const int n3 = c.n3;
    double *qa = x->Bv[0], *qb = x->Bv[1], *w = x->acc;
    if (!start) {
        launch_noise(x->dW, n3, seed, 0, 1.0, s);
        start = x->dW;
    }
    launch_lanczos_init(n3, start, qb, s);
    double *q = qb, *qp = qa;
    for (int j = 0; j < n_iter; ++j) {
        EpiArgs f{};
        f.mode = EPI_APPLY;
        f.m = 1;
        f.vout = w;
        product(x, q, 1, RPY_PREC_F64, f, s);
        launch_lanczos_step(n3, j, q, w, qp, c.lanc, s);
        double *t = q; q = qp; qp = t;   // qp now holds the old q, q the new one
    }
    int rc = check_launch("rpy_lanczos_bounds");
    if (rc) return rc;
    std::vector<double> ab(2 * n_iter), a(n_iter), b(n_iter);
    HIP_TRY(hipMemcpyAsync(ab.data(), c.lanc, sizeof(double) * 2 * n_iter,
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int j = 0; j < n_iter; ++j) {
        a[j] = ab[2 * j];
        b[j] = ab[2 * j + 1];
        if (alpha) alpha[j] = a[j];
        if (beta) beta[j] = b[j];
    }
    const double tmin = tridiag_eig(a.data(), b.data(), n_iter, 0);
    const double tmax = tridiag_eig(a.data(), b.data(), n_iter, n_iter - 1);
    const double rmin = fabs(b[n_iter - 1]) * tridiag_last(a.data(), b.data(), n_iter, tmin);
    const double rmax = fabs(b[n_iter - 1]) * tridiag_last(a.data(), b.data(), n_iter, tmax);
    double lo = (tmin - rmin) * (1.0 - margin);
    if (!(lo > 0)) lo = 0.5 * tmin;
    *d_min = lo;
    *d_max = (tmax + rmax) * (1.0 + margin);
    if (!isfinite(*d_min) || !isfinite(*d_max) || !(*d_max > *d_min)) return RPY_ENONFINITE;
    return RPY_OK;
}

extern "C" int chebyshev_sqrt_adaptive(rpy_ctx *x, const double *dw, double *out, int m,
                                       int n_start, int n_max, double d_min, double d_max,
                                       double tol, int prec, int *n_used, double *e_f,
                                       void *stream)
{
    if (!x || !dw || !out || !n_used || m < 1 || m > x->c.max_rhs || n_max < 2 ||
        n_max > x->c.cheb_keep || !(tol > 0) || !(d_min > 0) || !(d_max > d_min) ||
        !isfinite(d_max) || !prec_ok(x->c, prec))
        return RPY_EINVAL;
    hipStream_t s = S(stream);
    Ctx &c = x->c;
    const int floor_n = n_start >= 2 ? n_start : 0;
    launch_copy(c.vhist, dw, (size_t)m * c.n3, s);   // V_0
    launch_cheb_coeffs(c, 0, RPY_BOUNDS_EXPLICIT, 0.0, d_min, d_max, nullptr, s, floor_n, n_max);
    cheb_adapt_run(x, m, prec, 1, adapt_first(floor_n, d_min, d_max, n_max), n_max, tol, out,
                   e_f ? e_f : c.red, s);
    int rc = check_launch("chebyshev_sqrt_adaptive");
    if (rc) return rc;
    return adapt_result(x, n_used, s);
}

// Chebyshev recurrence on dw keeping every V_p (V_p at vh + p * ps), out =
// the sum with the coefficients in c.scal.
static void cheb_keep_run(rpy_ctx *x, const double *dw, double *vh, size_t ps, double *out,
                          int n_cheb, hipStream_t s)
{
    const Ctx &c = x->c;
    launch_copy(vh, dw, (size_t)c.n3, s);
    for (int p = 1; p < n_cheb; ++p) {
        EpiArgs f{};
        f.m = 1;
        f.p = p;
        f.scal = c.scal;
        f.acc = out;
        f.vout = vh + p * ps;
        f.vprev = vh + (p - 1) * ps;
        if (p == 1) {
            f.mode = EPI_CHEB_FIRST;
            f.dv = x->ddw;
        } else {
            f.mode = EPI_CHEB_NEXT;
            f.vprev2 = vh + (p - 2) * ps;
        }
        product(x, f.vprev, 1, RPY_PREC_F64, f, s);
    }
}

static int check_u_args(const rpy_ctx *x, int n_cheb, double d_min, double d_max)
{
    if (n_cheb < 2 || n_cheb > MAX_NCHEB || !(d_min > 0) || !(d_max > d_min) || !isfinite(d_max))
        return RPY_EINVAL;
    (void)x;
    return RPY_OK;
}

extern "C" int rpy_u_forward(rpy_ctx *x, const double *pos, const double *F, const double *dw,
                             int n_cheb, double d_min, double d_max, double *u, double *vh,
                             void *stream)
{
    if (!x || !pos || !F || !dw || !u) return RPY_EINVAL;
    int rc = check_u_args(x, n_cheb, d_min, d_max);
    if (rc) return rc;
    hipStream_t s = S(stream);
    Ctx &c = x->c;
    const size_t nv = (size_t)c.n3;
    launch_wrap_tables(c, pos, s);
    ++x->wrap_gen;
    launch_build_tiles(c, s);
    EpiArgs f{};
    f.mode = EPI_APPLY;
    f.m = 1;
    f.vout = x->Y;
    product(x, F, 1, RPY_PREC_F64, f, s);
    launch_cheb_coeffs(c, n_cheb, RPY_BOUNDS_EXPLICIT, 0.0, d_min, d_max, nullptr, s);
    if (vh) cheb_keep_run(x, dw, vh, nv, x->acc, n_cheb, s);
    else cheb_run(x, dw, x->acc, 1, n_cheb, RPY_PREC_F64, s);
    launch_add(u, x->Y, x->acc, nv, s);
    return check_launch("rpy_u_forward");
}

extern "C" int rpy_u_vjp(rpy_ctx *x, const double *pos, const double *F, const double *dw,
                         const double *vh, const double *g, int n_cheb, double d_min,
                         double d_max, double *g_pos, double *g_F, void *stream)
{
    if (!x || !pos || !F || !dw || !g || !g_pos) return RPY_EINVAL;
    Ctx &c = x->c;
    if (!c.grad) {
        snprintf(g_err, sizeof g_err, "context was created without grad");
        return RPY_EINVAL;
    }
    int rc = check_u_args(x, n_cheb, d_min, d_max);
    if (rc) return rc;
    if (n_cheb > c.cheb_keep) {
        snprintf(g_err, sizeof g_err, "n_cheb exceeds cheb_keep");
        return RPY_EINVAL;
    }
    hipStream_t s = S(stream);
    const size_t nv = (size_t)c.n3;
    launch_wrap_tables(c, pos, s);
    ++x->wrap_gen;
    launch_build_tiles(c, s);
    launch_cheb_coeffs(c, n_cheb, RPY_BOUNDS_EXPLICIT, 0.0, d_min, d_max, nullptr, s);
    size_t ps = nv;
    if (!vh) {   // recompute V_0 .. V_{n_cheb-1}
        ps = (size_t)c.rhs_cap * nv;
        cheb_keep_run(x, dw, c.vhist, ps, x->acc, n_cheb, s);
        vh = c.vhist;
    }
    EpiArgs f{};
    f.mode = EPI_APPLY;
    f.m = 1;
    f.vout = g_F ? g_F : x->Y;
    product(x, g, 1, RPY_PREC_F64, f, s);   // dL/dF = D g
    // pairs: x_0 = g, y_0 = F, y_q = V_{q-1}; x_q from the adjoint recurrence
    double *xy = c.xy;
    const int P = n_cheb;
    launch_copy(xy, g, nv, s);
    launch_copy(xy + nv, F, nv, s);
    for (int q = 1; q < P; ++q) launch_copy(xy + (2 * q + 1) * nv, vh + (q - 1) * ps, nv, s);
    double *mu[3] = {c.mur, c.mur + nv, c.mur + 2 * nv};
    launch_adj_init(c, P - 1, P - 1 == 1 ? 1.0 : 2.0, g, mu[(P - 1) % 3], xy + 2 * (P - 1) * nv, s);
    for (int p = P - 2; p >= 1; --p) {
        EpiArgs a{};
        a.mode = EPI_ADJ;
        a.m = 1;
        a.p = p;
        a.scal = c.scal;
        a.vprev = mu[(p + 1) % 3];
        a.vprev2 = p + 2 <= P - 1 ? mu[(p + 2) % 3] : nullptr;
        a.vout = mu[p % 3];
        a.acc = const_cast<double *>(g);
        a.dv = xy + 2 * p * nv;
        a.xs = p == 1 ? 1.0 : 2.0;
        product(x, a.vprev, 1, RPY_PREC_F64, a, s);
    }
    launch_grad_wtiles(c, P, s);
    launch_grad_real(c, s);
    const int qg = c.rhs_cap / 2;
    for (int q0 = 0; q0 < P; q0 += qg) {
        const int nq = P - q0 < qg ? P - q0 : qg;
        launch_grad_sf(c, xy + 2 * q0 * nv, 2 * nq, s);
        launch_sf_reduce(c, 2 * nq, s);
        launch_grad_kspace(c, xy + 2 * q0 * nv, nq, q0 > 0, s);
    }
    launch_grad_sum(c, g_pos, s);
    return check_launch("rpy_u_vjp");
}

extern "C" int rpy_bounds(rpy_ctx *x, int rule, double C, double *d_min, double *d_max,
                          void *stream)
{
    if (!x || !d_min || !d_max) return RPY_EINVAL;
    if (rule == RPY_BOUNDS_PAPER) {
        if (!(C > 0) || !isfinite(C)) return RPY_EINVAL;
    } else if (rule != RPY_BOUNDS_DILUTE) {
        return RPY_EINVAL;
    }
    hipStream_t s = S(stream);
    const Ctx &c = x->c;
    const size_t nv = (size_t)c.n3;
    // [U+] for the paper's rule; [U+, U-] side by side for the dilute rule
    const int m = rule == RPY_BOUNDS_DILUTE ? 2 : 1;
    const double *v = x->F + nv;
    if (m == 2) {
        launch_copy(x->Bv[0], x->F + nv, nv, s);
        launch_copy(x->Bv[0] + nv, x->Um, nv, s);
        v = x->Bv[0];
    }
    EpiArgs f{};
    f.mode = EPI_APPLY;
    f.m = m;
    f.vout = x->Y + nv;
    product(x, v, m, RPY_PREC_F64, f, s);
    launch_cheb_coeffs(c, 2, rule, C, 0, 0, x->Y + nv, s);
    int rc = check_launch("rpy_bounds");
    if (rc) return rc;
    double h[2];
    HIP_TRY(hipMemcpyAsync(h, c.scal, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int fl = 0;
    HIP_TRY(hipMemcpy(&fl, c.flags, sizeof fl, hipMemcpyDeviceToHost));
    *d_min = h[0];
    *d_max = h[1];
    return fl ? RPY_ENONFINITE : RPY_OK;
}

// Springs plus excluded volume; `rt` holds the wrapped positions of `pos`.
static int forces(rpy_ctx *x, const double *pos, const double *rt, double zstar, double dstar,
                  double rcut, double *F, hipStream_t s)
{
    Ctx &c = x->c;
    launch_spring_forces(c, pos, F, s);
    if (zstar > 0) {
        const int nc = (int)floor(c.L / rcut);
        c.ncell = nc >= 3 ? (nc > 64 ? 64 : nc) : 0;
        launch_cell_list(c, rt, rcut, s);
        launch_ev_forces(c, rt, zstar, dstar, rcut, F, s);
    }
    return RPY_OK;
}

static int check_ev(const Ctx &c, double zstar, double dstar, double rcut)
{
    if (zstar < 0 || !isfinite(zstar)) return RPY_EINVAL;
    if (zstar > 0 && (!(dstar > 0) || !(rcut > 0) || !(rcut < 0.5 * c.L))) {
        snprintf(g_err, sizeof g_err, "excluded volume needs d* > 0 and 0 < rcut < L/2");
        return RPY_EINVAL;
    }
    return RPY_OK;
}

extern "C" int rpy_forces(rpy_ctx *x, const double *pos, double zstar, double dstar,
                          double rcut, double *out, void *stream)
{
    if (!x || !pos || !out) return RPY_EINVAL;
    int rc = check_ev(x->c, zstar, dstar, rcut);
    if (rc) return rc;
    hipStream_t s = S(stream);
    // its own wrapped copy: the tables of the built D stay untouched
    if (zstar > 0) launch_wrap_positions(x->c, pos, x->c.rt_ev, s);
    forces(x, pos, x->c.rt_ev, zstar, dstar, rcut, out, s);
    return check_launch("rpy_forces");
}

extern "C" int rpy_forces_vjp(rpy_ctx *x, const double *pos, double zstar, double dstar,
                              double rcut, const double *gF, double *g_pos, void *stream)
{
    if (!x || !pos || !gF || !g_pos) return RPY_EINVAL;
    int rc = check_ev(x->c, zstar, dstar, rcut);
    if (rc) return rc;
    hipStream_t s = S(stream);
    Ctx &c = x->c;
    launch_spring_forces(c, gF, g_pos, s);   // the spring operator is linear and symmetric
    if (zstar > 0) {
        launch_wrap_positions(c, pos, c.rt_ev, s);
        const int nc = (int)floor(c.L / rcut);
        c.ncell = nc >= 3 ? (nc > 64 ? 64 : nc) : 0;
        launch_cell_list(c, c.rt_ev, rcut, s);
        launch_ev_vjp(c, c.rt_ev, zstar, dstar, rcut, gF, g_pos, s);
    }
    return check_launch("rpy_forces_vjp");
}

extern "C" int bd_step(rpy_ctx *x, double *pos, const bd_params *bp, const double *dw,
                       uint64_t seed, uint64_t step, double *drift, double *noise,
                       double *e_f, void *stream)
{
    if (!x || !pos || !bp) return RPY_EINVAL;
    Ctx &c = x->c;
    const bool adapt = bp->tol > 0;
    if (!(bp->dt > 0) || !isfinite(bp->dt) || !prec_ok(c, bp->prec) || !(bp->tol == bp->tol) ||
        bp->tol == INFINITY)
        return RPY_EINVAL;
    if (adapt) {
        if (bp->n_max < 2 || bp->n_max > MAX_NCHEB || bp->n_max > c.cheb_keep) {
            snprintf(g_err, sizeof g_err, "the adaptive order needs 2 <= n_max <= cheb_keep");
            return RPY_EINVAL;
        }
    } else if (bp->n_cheb < 2 || bp->n_cheb > MAX_NCHEB) {
        return RPY_EINVAL;
    }
    const int rule = bp->bounds_rule;
    if (rule == RPY_BOUNDS_EXPLICIT) {
        if (!(bp->d_min > 0) || !(bp->d_max > bp->d_min) || !isfinite(bp->d_max))
            return RPY_EINVAL;
    } else if (rule == RPY_BOUNDS_PAPER) {
        if (!(bp->bounds_C > 0) || !isfinite(bp->bounds_C)) return RPY_EINVAL;
    } else if (rule != RPY_BOUNDS_DILUTE) {
        return RPY_EINVAL;
    }
    int rc = check_ev(c, bp->ev_zstar, bp->ev_dstar, bp->ev_rcut);
    if (rc) return rc;
    hipStream_t s = S(stream);
    const size_t nv = (size_t)c.n3;
    launch_wrap_tables(c, pos, s);
    ++x->wrap_gen;
    // The first Chebyshev product rides with the drift product: one FP64
    // pass over D for [F, U+, (U-,) dW], then the coefficients, then V_1
    // from D.dW; the products from V_1 on take bp->prec.  D.dW in FP64 also
    // makes E_f measure the square root against the FP64 quadratic form.
    double *w = x->F + 2 * nv;
    // forces and noise on the side stream, beside the build
    HIP_TRY(hipEventRecord(x->fork, s));
    HIP_TRY(hipStreamWaitEvent(x->side, x->fork, 0));
    {
        ProfScope ps(x, RPY_PROF_OTHER, x->side);
        forces(x, pos, c.rt, bp->ev_zstar, bp->ev_dstar, bp->ev_rcut, x->F, x->side);
        if (!dw) launch_noise(w, (int64_t)nv, seed, step, bp->dt, x->side);
        else launch_copy(w, dw, nv, x->side);
    }
    HIP_TRY(hipEventRecord(x->join, x->side));
    {
        ProfScope ps(x, RPY_PROF_BUILD, s);
        launch_build_tiles(c, s);
    }
    HIP_TRY(hipStreamWaitEvent(s, x->join, 0));
    // the drift product: F, then U+ (paper and dilute rules) and U- (dilute),
    // then dW; D.F lands in Y, D.U+ in Y + nv, D.dW last
    const int nb = rule == RPY_BOUNDS_PAPER ? 1 : rule == RPY_BOUNDS_DILUTE ? 2 : 0;
    EpiArgs f{};
    f.mode = EPI_APPLY;
    f.vout = x->Y;
    f.m = 2 + nb;
    if (nb == 1) {
        product(x, x->F, f.m, RPY_PREC_F64, f, s);   // [F, U+, dW] contiguous
    } else {
        double *g = x->Bv[0];   // free until the recurrence's second product
        launch_copy(g, x->F, nv, s);
        if (nb == 2) {
            launch_copy(g + nv, x->F + nv, nv, s);
            launch_copy(g + 2 * nv, x->Um, nv, s);
        }
        launch_copy(g + (1 + nb) * nv, w, nv, s);
        product(x, g, f.m, RPY_PREC_F64, f, s);
    }
    const double *du = x->Y + nv;
    const int floor_n = adapt ? (bp->n_cheb >= 2 ? bp->n_cheb : 0) : -1;
    const int nmax = adapt ? bp->n_max : bp->n_cheb;
    launch_cheb_coeffs(c, bp->n_cheb, rule, bp->bounds_C, bp->d_min, bp->d_max,
                       nb ? du : nullptr, s, floor_n, nmax);
    if (adapt) {
        const size_t ps = (size_t)c.rhs_cap * nv;
        launch_copy(c.vhist, w, nv, s);   // V_0
        // The first order the device can start from.  Explicit interval: the
        // device's own value.  The paper's rule fixes d_max / d_min = C N^0.6
        // whatever D is, so eq. nint is known up to the rounding of that
        // ratio: one order below it is safe (a trial below the device's first
        // order returns at once).  The dilute rule: from the lowest order.
        int host_first = floor_n >= 2 ? (floor_n < nmax ? floor_n : nmax) : 2;
        if (rule == RPY_BOUNDS_EXPLICIT) {
            host_first = adapt_first(floor_n, bp->d_min, bp->d_max, nmax);
        } else if (rule == RPY_BOUNDS_PAPER && floor_n < 2) {
            const int k = adapt_first(0, 1.0, bp->bounds_C * pow((double)c.N, 0.6), nmax) - 1;
            host_first = k < 2 ? 2 : k;
        }
        launch_cheb_first(c, x->Y + (1 + nb) * nv, w, c.vhist + ps, x->acc, x->ddw, s);
        cheb_adapt_run(x, 1, bp->prec, 2, host_first, nmax, bp->tol, x->dS,
                       e_f ? e_f : c.red, s);
    } else {
        launch_cheb_first(c, x->Y + (1 + nb) * nv, w, x->Bv[1], x->dS, x->ddw, s);
        cheb_run(x, w, x->dS, 1, bp->n_cheb, bp->prec, s, 2);
        if (e_f) launch_sqrt_error(c, 1, w, x->ddw, x->dS, e_f, s);
    }
    if (drift) launch_copy(drift, x->Y, nv, s);
    if (noise) launch_copy(noise, x->dS, nv, s);
    launch_euler(c, pos, bp->dt, x->Y, x->dS, s);
    return check_launch("bd_step");
}

extern "C" int rpy_status(rpy_ctx *x, void *stream)
{
    if (!x) return RPY_EINVAL;
    HIP_TRY(hipStreamSynchronize(S(stream)));
    int fl = 0;
    HIP_TRY(hipMemcpy(&fl, x->c.flags, sizeof fl, hipMemcpyDeviceToHost));
    if (fl) {
        HIP_TRY(hipMemset(x->c.flags, 0, sizeof(int)));
        snprintf(g_err, sizeof g_err, "non-finite position");
        return RPY_ENONFINITE;
    }
    long long etol = 0;
    HIP_TRY(hipMemcpy(&etol, &x->c.adapt->etol, sizeof etol, hipMemcpyDeviceToHost));
    if (etol) {
        HIP_TRY(hipMemset(&x->c.adapt->etol, 0, sizeof etol));
        return RPY_ETOL;
    }
    return RPY_OK;
}

extern "C" int rpy_order_stats(rpy_ctx *x, int64_t *calls, double *mean_order, int *max_order,
                               int64_t *missed, void *stream)
{
    if (!x || !calls || !mean_order || !max_order || !missed) return RPY_EINVAL;
    AdaptState st;
    HIP_TRY(hipMemcpyAsync(&st, x->c.adapt, sizeof st, hipMemcpyDeviceToHost, S(stream)));
    HIP_TRY(hipStreamSynchronize(S(stream)));
    *calls = st.calls;
    *mean_order = st.calls ? (double)st.sum_orders / (double)st.calls : 0.0;
    *max_order = st.max_order;
    *missed = st.missed;
    AdaptState z = st;
    z.calls = z.sum_orders = z.missed = 0;
    z.max_order = 0;
    HIP_TRY(hipMemcpy(x->c.adapt, &z, sizeof z, hipMemcpyHostToDevice));
    return RPY_OK;
}

extern "C" int rpy_real_space_dense(rpy_ctx *x, double *out, void *stream)
{
    if (!x || !out) return RPY_EINVAL;
    if (x->c.lma) {
        snprintf(g_err, sizeof g_err, "the low-memory form stores no real-space matrix");
        return RPY_EINVAL;
    }
    launch_dense_copy(x->c, out, S(stream));
    return check_launch("rpy_real_space_dense");
}

extern "C" int rpy_observables(rpy_ctx *x, const double *pos, double *re2, double *rg2,
                               void *stream)
{
    if (!x || !pos || !re2 || !rg2) return RPY_EINVAL;
    launch_observables(x->c, pos, re2, rg2, S(stream));
    return check_launch("rpy_observables");
}

extern "C" int rpy_gaussian_noise(double *out, int64_t count, uint64_t seed, uint64_t step,
                                  double dt, void *stream)
{
    if (!out || count < 0 || !(dt > 0)) return RPY_EINVAL;
    launch_noise(out, count, seed, step, dt, S(stream));
    return check_launch("rpy_gaussian_noise");
}

extern "C" int rpy_philox4x32_10(const uint32_t *ck, uint32_t *out, int64_t n, void *stream)
{
    if (!ck || !out || n < 0) return RPY_EINVAL;
    launch_philox(ck, out, n, S(stream));
    return check_launch("rpy_philox4x32_10");
}

extern "C" int rpy_host_pair_block(const rpy_params *p, const double *d, int self, double *out)
{
    int n2 = 0;
    if (!d || !out) return RPY_EINVAL;
    int rc = validate(p, &n2);
    if (rc) return rc;
    const PairConst pc = make_pair_const(p->box_l, p->a, p->alpha, p->r_c);
    double b[6];
    pair_block(d[0], d[1], d[2], self != 0, pc, b);
    const double v[9] = {b[0], b[1], b[2], b[1], b[3], b[4], b[2], b[4], b[5]};
    memcpy(out, v, sizeof v);
    return RPY_OK;
}

extern "C" int rpy_profile_enable(rpy_ctx *x, int cap)
{
    if (!x || cap < 0) return RPY_EINVAL;
    Prof &p = x->prof;
    if (cap > p.alloc) {
        for (int k = 0; k < RPY_PROF_KINDS; ++k) {
            hipEvent_t *ev = new (std::nothrow) hipEvent_t[2 * (size_t)cap];
            if (!ev) return RPY_ENOMEM;
            for (int i = 0; i < 2 * p.alloc; ++i) ev[i] = p.ev[k][i];
            for (int i = 2 * p.alloc; i < 2 * cap; ++i) HIP_TRY(hipEventCreate(&ev[i]));
            delete[] p.ev[k];
            p.ev[k] = ev;
        }
        p.alloc = cap;
    }
    p.cap = cap;
    for (int k = 0; k < RPY_PROF_KINDS; ++k) p.n[k] = 0;
    return RPY_OK;
}

extern "C" int rpy_profile_read(rpy_ctx *x, int kind, int64_t *count, double *total_ms)
{
    if (!x || kind < 0 || kind >= RPY_PROF_KINDS || !count || !total_ms) return RPY_EINVAL;
    HIP_TRY(hipDeviceSynchronize());
    Prof &p = x->prof;
    double t = 0.0;
    for (int i = 0; i < p.n[kind]; ++i) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, p.ev[kind][2 * i], p.ev[kind][2 * i + 1]));
        t += ms;
    }
    *count = p.n[kind];
    *total_ms = t;
    p.n[kind] = 0;
    return RPY_OK;
}

extern "C" int rpy_num_kvectors(const rpy_ctx *x) { return x ? x->c.nk : -1; }

extern "C" const char *rpy_strerror(int code)
{
    switch (code) {
    case RPY_OK: return "ok";
    case RPY_EINVAL: return g_err[0] ? g_err : "invalid argument";
    case RPY_EGEOM: return "box too small for the bead radius (need 4a < L)";
    case RPY_ENONFINITE: return "non-finite position";
    case RPY_ETOL: return "square-root error estimate above tolerance";
    case RPY_ENOMEM: return g_err[0] ? g_err : "device allocation failed";
    case RPY_EHIP: return g_err[0] ? g_err : "HIP runtime error";
    default: return "unknown error";
    }
}
