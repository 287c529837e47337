/*
 * rpy.h -- C ABI of librpy, the MI355X (gfx950) implementation of the
 * Ewald-summed Rotne-Prager-Yamakawa Brownian-dynamics step of
 * Jain, Sunthar, Duenweg & Prakash, arXiv:1203.6208.
 *
 * Conventions for every entry point:
 *  - Array arguments are DEVICE pointers to caller-owned memory unless a
 *    comment says "host".  The library never frees or retains them past the
 *    call (work is enqueued on the stream; the caller must keep the memory
 *    alive until the stream reaches that point).
 *  - All floating-point arrays are IEEE binary64, C-contiguous.
 *  - Positions are [N][3] (bead nu at offset 3*nu).  Vectors are [m][N][3]:
 *    right-hand side j starts at offset 3*N*j and component i of bead nu is at
 *    3*nu + i within it (the flattened block index of the section "Governing
 *    equation").  Positions are unwrapped; the library wraps them itself.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Calls only enqueue
 *    work on it and do not synchronise, unless a comment says "synchronises".
 *  - Return value: RPY_OK (0) or a negative RPY_E* code.  An error detected
 *    on the host leaves outputs untouched.  A non-finite position is detected
 *    on the device; it is reported by the next synchronising call
 *    (rpy_status, rpy_bounds) as RPY_ENONFINITE.
 *  - A context is not thread-safe: calls on one context must be ordered on a
 *    single stream by the caller.  Distinct contexts are independent.
 */
#ifndef RPY_H
#define RPY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    RPY_OK = 0,
    RPY_EINVAL = -1,     /* invalid argument (sizes, parameters, null pointers) */
    RPY_EGEOM = -2,      /* box too small for the bead radius: 4a >= L */
    RPY_ENONFINITE = -3, /* NaN or Inf found in positions */
    RPY_ETOL = -4,       /* square-root error estimate above the tolerance */
    RPY_ENOMEM = -5,     /* device allocation failed in rpy_create */
    RPY_EHIP = -6        /* a HIP runtime call failed; see rpy_strerror */
};

/* Arithmetic of the real-space D.V products (the k-space sums, the
 * Chebyshev recurrence and all accumulation across tiles stay FP64). */
enum { RPY_PREC_F64 = 0, RPY_PREC_F32 = 1, RPY_PREC_BF16 = 2 };

/* Chebyshev interval (section "Decomposition of the diffusion tensor"):
 *  RPY_BOUNDS_EXPLICIT  the caller's [d_min, d_max];
 *  RPY_BOUNDS_PAPER     the paper's semidilute rule (eq. lmax-lmin-dilute,
 *                       fmax, fmin): lmax = 0.35 N^0.6 U+.D.U+/(3N),
 *                       d_max = lmax, d_min = lmax / (C N^0.6);
 *  RPY_BOUNDS_DILUTE    the dilute rule of eq. lmax-lmin-dilute with the
 *                       factors the paper quotes for it: d_max = 2 U+.D.U+/(3N),
 *                       d_min = U-.D.U-/(2 3N), U+ all ones, U- alternating
 *                       +1, -1 over the flattened index 3 nu + i.
 * The rules cost one FP64 product with U+ (and U-). */
enum { RPY_BOUNDS_EXPLICIT = 0, RPY_BOUNDS_PAPER = 1, RPY_BOUNDS_DILUTE = 2 };

/* Problem statement (sections "Governing equation" and "Implementation of
 * the Ewald sum"): N beads in a cubic periodic box of side box_l; bead radius
 * a = sqrt(pi) h*; Ewald parameter alpha; real-space cutoff r_c (a periodic
 * image enters the real-space sum iff |r| <= r_c); reciprocal cutoff k_c
 * (the wave vectors are k = 2 pi n / L with n integer, n != 0 and
 * |n|^2 <= floor((k_c L / (2 pi))^2)).  Beads are stored chain after chain,
 * beads_per_chain each (n_chains * beads_per_chain == n_beads). */
typedef struct {
    int32_t n_beads;
    int32_t n_chains;
    int32_t beads_per_chain;
    int32_t lowp;      /* low-precision copy of D kept by rpy_ewald_build:
                          RPY_PREC_F64 (none), RPY_PREC_F32 or RPY_PREC_BF16 */
    int32_t max_rhs;   /* largest m accepted by rpy_apply/chebyshev_sqrt_apply
                          (1..16); with max_rhs >= 5 (and lma = 0) the
                          context also holds the buffers of the matrix-core
                          block product (per-tile FP64 partial sums and the
                          structure-factor phases: about 150 MB at N = 4000) */
    int32_t cheb_keep; /* Chebyshev vectors V_p kept for the adaptive order
                          (bd_step and chebyshev_sqrt_apply with tol > 0,
                          chebyshev_sqrt_adaptive) and rpy_u_vjp: the largest
                          order those calls may use (0 disables them; at most
                          512); cheb_keep x max(max_rhs, 4) x 3N doubles */
    int32_t grad;      /* 1: also hold the buffers of rpy_u_vjp (a W
                          matrix on the upper tiles, row-major, about
                          9N^2/2 doubles, and 2 cheb_keep + 4 vectors of
                          3N); needs cheb_keep >= 2 and lma = 0.  0: none */
    int32_t lma;       /* 0: high-memory form, the real-space part of D is
                          stored (upper tiles, the 6 distinct entries of
                          each symmetric 3 x 3 bead-pair block: about
                          3N(N+1) doubles, read by every product of any
                          number of vectors).
                          1: low-memory form (section "Low memory
                          algorithm"): nothing of size N^2 is stored; every
                          product recomputes the real-space sum over a cell
                          list of side >= max(r_c, 2a), which needs
                          max(r_c, 2a) <= L/3; FP64 only (lowp is ignored),
                          no rpy_real_space_dense, no grad */
    double box_l;
    double a;
    double alpha;
    double r_c;
    double k_c;
} rpy_params;

typedef struct rpy_ctx rpy_ctx;

/* Validate p and allocate every device buffer the context needs (the stored
 * real-space matrix, phase tables, work space).  No later call allocates.
 * Errors: RPY_EINVAL for n_beads <= 0, box_l <= 0, a <= 0, alpha <= 0,
 * r_c <= 0, k_c <= 0, an empty wave-vector set, chains that do not tile the
 * beads, max_rhs outside 1..16 or an unknown lowp; RPY_EGEOM if 4a >= L
 * (then two images of one pair could overlap); RPY_ENOMEM, RPY_EHIP. */
int rpy_create(rpy_ctx **out, const rpy_params *p);

/* Free the context and its device memory (synchronises the device). */
void rpy_destroy(rpy_ctx *c);

/* Build the diffusion tensor for the positions pos [N][3] (device):
 * wraps positions into the box, tabulates the per-bead Fourier phases, and
 * writes the real-space part of D -- self term, the lattice sum of M1 over
 * every image with |r| <= r_c and the overlap correction M* for every image
 * with |r| < 2a (eq. DFmodified; the reciprocal sum taken with
 * cos(k.(r_nu - r_mu)), M* as the branch-B minus branch-A difference) --
 * into the context's symmetric tile storage (plus the low-precision copy if
 * lowp is set).  The reciprocal-space part is applied per product
 * (rpy_apply), as in the paper's high-memory algorithm (section "Optimisation
 * of each Euler time step"). */
int rpy_ewald_build(rpy_ctx *c, const double *pos, void *stream);

/* out = D . v for m right-hand sides (v, out: device [m][N][3], not
 * aliased), D being the full periodic diffusion tensor of the last build:
 * the stored real-space part in arithmetic `prec` (RPY_PREC_*; FP32/BF16 need
 * the matching lowp copy) plus the reciprocal-space sum in FP64 (eq.
 * DFmodified).  With 5 <= m <= 16 (max_rhs >= 5) the real-space part runs on
 * the matrix cores straight from the packed tile planes: FP64 tiles on the
 * FP64 matrix cores with FP64 accumulation, FP32 tiles with FP32
 * accumulation inside each 64-bead tile, BF16 tiles likewise (the vectors
 * enter as a hi + lo BF16 pair, so only D is rounded to BF16); the
 * reciprocal sum and the sums over tiles stay FP64.  Results are
 * deterministic run to run.  Errors: RPY_EINVAL (m outside 1..max_rhs, prec
 * not built, null pointers). */
int rpy_apply(rpy_ctx *c, const double *v, double *out, int m, int prec,
              void *stream);

/* Chebyshev interval by rule (RPY_BOUNDS_PAPER with constant C, or
 * RPY_BOUNDS_DILUTE, C unused) from the last build: one FP64 product with U+
 * (and U-).  d_min, d_max: HOST outputs.  Synchronises the stream; returns
 * RPY_EINVAL for another rule or C <= 0 with the paper's rule, and
 * RPY_ENONFINITE if the last build saw a non-finite position. */
int rpy_bounds(rpy_ctx *c, int rule, double C, double *d_min, double *d_max,
               void *stream);

/* Fixman-Chebyshev Brownian term (section "Decomposition of the diffusion
 * tensor", eq. cheb1-cheb3): out = sum_{p<N_Ch} c_p V_p - (c_0/2) dW with
 * V_0 = dW, V_1 = Y V_0, V_p = 2 Y V_{p-1} - V_{p-2},
 * Y = (2 D - (d_max + d_min) I) / (d_max - d_min), c_p the coefficients of
 * the interpolant of sqrt at the N_Ch Chebyshev-Gauss nodes of
 * [d_min, d_max].  dw, out: device [m][N][3], not aliased.  The N_Ch - 1
 * products use `prec` for the stored real-space part.
 *  tol <= 0: N_Ch = n_cheb.
 *  tol > 0: the paper's adaptive order (eq. nint, then the E_f criterion):
 *    N_Ch starts at nint(sqrt(d_max/d_min)) + 1 (rounded half away from zero,
 *    at least 2) and grows by one term -- one more product and a new sum of
 *    the kept V_p with the coefficients of the new order -- until
 *    E_f < tol for every right-hand side, or N_Ch = n_cheb, the largest order
 *    tried (needs cheb_keep >= n_cheb).  The whole search is enqueued at once;
 *    on the device the products and sums past the settled order return at
 *    once, so the call does not synchronise unless n_used is requested.  A
 *    tolerance still missed at n_cheb is reported as RPY_ETOL by this call
 *    when n_used is given, else by the next rpy_status (outputs written).
 * n_used: optional HOST output, the N_Ch used (synchronises the stream when
 * tol > 0).  e_f: optional device [m] output of the error estimate
 * E_f = sqrt(|dS.dS - dW.D.dW| / dW.D.dW) per right-hand side.
 * Errors: RPY_EINVAL for n_cheb < 2, d_min <= 0, d_min >= d_max, m outside
 * 1..max_rhs, prec not built, a non-finite tol, or tol > 0 with
 * n_cheb > cheb_keep. */
int chebyshev_sqrt_apply(rpy_ctx *c, const double *dw, double *out, int m,
                         int n_cheb, double d_min, double d_max, double tol,
                         int prec, int *n_used, double *e_f, void *stream);

/* Eigenvalue bounds of D of the last build by the Lanczos recurrence in FP64
 * (the interval of eq. cheb3 must satisfy d_max >= lambda_max and
 * d_min <= lambda_min, section "Decomposition of the diffusion tensor"):
 *   q_1 = r/|r|,  w = D q_j - beta_{j-1} q_{j-1},  alpha_j = q_j.w,
 *   w -= alpha_j q_j,  beta_j = |w|,  q_{j+1} = w/beta_j,   j = 1..n_iter
 * (one FP64 product per step, no reorthogonalisation).  r is `start`
 * (device [N][3]) or, if NULL, Gaussian noise from (seed, step 0) as in
 * rpy_gaussian_noise.  From the extreme eigenvalues theta of the tridiagonal
 * T and their residual bounds res = beta_n |s_n| (s the unit eigenvector):
 *   d_min = (theta_min - res_min)(1 - margin),
 *   d_max = (theta_max + res_max)(1 + margin)
 * (d_min = theta_min/2 if that is not positive).  d_min, d_max: HOST outputs;
 * alpha, beta: optional HOST [n_iter] outputs.  Synchronises the stream.
 * Errors: RPY_EINVAL for n_iter outside 2..2048, margin < 0 or null outputs. */
int rpy_lanczos_bounds(rpy_ctx *c, int n_iter, uint64_t seed, const double *start,
                       double margin, double *d_min, double *d_max, double *alpha,
                       double *beta, void *stream);

/* The adaptive order of chebyshev_sqrt_apply with an explicit first order:
 * N_Ch starts at n_start (or, if n_start < 2, at eq. nint) and grows by one
 * term until E_f < tol for every right-hand side or N_Ch = n_max.  n_used:
 * HOST output, the final N_Ch; e_f: optional device [m] output.  Synchronises
 * the stream once, at the end.  Needs cheb_keep >= n_max.  Returns RPY_ETOL
 * (outputs written) if E_f >= tol at n_max; RPY_EINVAL as
 * chebyshev_sqrt_apply, for tol <= 0, or n_max outside 2..cheb_keep. */
int chebyshev_sqrt_adaptive(rpy_ctx *c, const double *dw, double *out, int m,
                            int n_start, int n_max, double d_min, double d_max,
                            double tol, int prec, int *n_used, double *e_f,
                            void *stream);

/* One Euler-Maruyama step (eq. sde with kappa = 0):
 *   r <- r + (dt/4) D.F + (1/sqrt 2) dS,  dS ~ sqrt(D) dW by Chebyshev,
 * with F = Hookean springs (F_mu = Q_mu - Q_{mu-1}) plus, when ev_zstar > 0,
 * narrow-Gaussian excluded volume between all beads,
 *   U = zs ds^-3 exp(-r^2 / (2 ds^2)) with zs = ev_zstar, ds = ev_dstar,
 * for pairs closer than ev_rcut
 * (minimum image; requires ev_rcut < L/2).
 * dw: device [N][3] noise with variance dt, or NULL to draw it on the device
 * from (seed, step) with Philox4x32-10 and Box-Muller (the mapping of
 * rpy_gaussian_noise with count 3N).
 * pos: device [N][3], updated in place.  drift, noise, e_f: optional device
 * outputs ([N][3] D.F, [N][3] dS, [1] E_f).  The interval follows
 * bounds_rule, computed on the device from this step's D.
 * Order: tol <= 0 takes N_Ch = n_cheb.  tol > 0 takes the paper's adaptive
 * order as chebyshev_sqrt_apply does -- N_Ch starts at n_cheb if >= 2, else at
 * eq. nint on this step's interval, and grows by one term until E_f < tol or
 * N_Ch = n_max (needs 2 <= n_max <= cheb_keep) -- with no host
 * synchronisation; a missed tolerance is counted and reported as RPY_ETOL by
 * rpy_status, and rpy_order_stats reports the orders used.
 * prec selects the arithmetic of the Chebyshev products from V_1 on; the
 * drift, the bounds and the first product D.dW (taken in the same FP64 pass
 * over D as D.F, and reused by E_f) always use FP64.  The forces and the device noise run on a second
 * stream owned by the context, forked from `stream` after the wrap and
 * joined back before the drift product (event record / wait, no host
 * synchronisation), so that they overlap the tile build; everything the call
 * enqueues is ordered before later work on `stream`.
 * Errors: RPY_EINVAL for dt <= 0, an unknown rule, C <= 0 with the paper's
 * rule, an invalid explicit interval, n_cheb outside 2..512 with tol <= 0,
 * n_max outside 2..cheb_keep with tol > 0, prec not built, or invalid
 * excluded-volume parameters (ev_zstar > 0 needs ev_dstar > 0 and
 * 0 < ev_rcut < L/2). */
typedef struct {
    double dt;
    double ev_zstar;    /* 0 disables excluded volume */
    double ev_dstar;
    double ev_rcut;
    double bounds_C;    /* C of the paper's rule */
    double d_min;       /* explicit bounds (RPY_BOUNDS_EXPLICIT) */
    double d_max;
    double tol;         /* E_f tolerance of the adaptive order; <= 0: fixed order */
    int32_t n_cheb;     /* fixed N_Ch; with tol > 0 the first order (< 2: eq. nint) */
    int32_t bounds_rule;
    int32_t prec;
    int32_t n_max;      /* with tol > 0: the largest N_Ch tried */
} bd_params;

int bd_step(rpy_ctx *c, double *pos, const bd_params *bp, const double *dw,
            uint64_t seed, uint64_t step, double *drift, double *noise,
            double *e_f, void *stream);

/* ------------------------------------------------------------------------
 * Differentiation.  u(R, F) = D(R) F + p(D(R)) dW, where p(D) dW is the
 * n_cheb-term Chebyshev sum of chebyshev_sqrt_apply on the fixed interval
 * [d_min, d_max] (eq. DF and eq. cheb1-cheb3; the interval is an input, so
 * no derivative flows through it).  The derivatives of D's pair terms are
 * those of eq. M1, b1/b2 and cor5 (with the readings of rpy_ewald_build) and
 * of the cosine of eq. M2; at r = 0 between distinct beads the pair term is
 * not differentiable and contributes nothing.
 *
 * rpy_u_forward: builds D at pos and writes u (device [N][3]).  vh:
 * optional device [n_cheb][N][3] that receives V_0 .. V_{n_cheb-1} of the
 * recurrence for a later rpy_u_vjp (NULL: not kept).
 *
 * rpy_u_vjp: for L = g . u (g device [N][3]) writes g_pos = dL/dR and, if
 * g_F is not NULL, g_F = dL/dF = D g (device [N][3] each).  vh: the V_p
 * written by rpy_u_forward for the same pos and dw, or NULL to recompute
 * them (then n_cheb <= cheb_keep).  Rebuilds D at pos.  The context must be
 * created with grad = 1 and n_cheb <= cheb_keep; otherwise RPY_EINVAL.
 * Cost: one build, n_cheb - 1 products (n_cheb - 1 more with vh = NULL),
 * one tile pass over a W matrix of the stored size, the real-space image
 * derivatives of every pair, and the structure factors of 2 n_cheb vectors. */
int rpy_u_forward(rpy_ctx *c, const double *pos, const double *F,
                  const double *dw, int n_cheb, double d_min, double d_max,
                  double *u, double *vh, void *stream);
int rpy_u_vjp(rpy_ctx *c, const double *pos, const double *F,
              const double *dw, const double *vh, const double *g, int n_cheb,
              double d_min, double d_max, double *g_pos, double *g_F,
              void *stream);

/* Transpose of the force Jacobian (forces as rpy_forces): g_pos = (dF/dR)^T
 * gF.  The spring part is the (symmetric) spring operator applied to gF; the
 * excluded-volume part adds sum_mu J(d) (gF_nu - gF_mu) with
 * J(d) = (zstar / dstar^5) exp(-|d|^2 / (2 dstar^2)) (I - d d^T / dstar^2),
 * minimum image, |d| <= rcut.  pos, gF, g_pos: device [N][3]. */
int rpy_forces_vjp(rpy_ctx *c, const double *pos, double zstar, double dstar,
                   double rcut, const double *gF, double *g_pos, void *stream);

/* rpy_forces without a context, for callers that cannot allocate device
 * memory (code under stream capture, tight stepping loops, harnesses that
 * forbid allocation): the same springs and narrow-Gaussian excluded volume
 * into out[N][3] (device), for N = n_chains x beads_per_chain beads in a box
 * of side box_l.  It allocates nothing: its scratch (wrapped positions, the
 * cell list, about 3.9 MB) is a static device array of the library, one per
 * GPU, looked up on the first call on that GPU and kept until the process
 * ends.  Every call on a GPU uses that GPU's one array, so calls that overlap
 * on one GPU (different streams or host threads) race; calls ordered on one
 * stream do not.  A non-finite position is not reported (the forces of its
 * chain come out non-finite).  Errors: RPY_EINVAL for n_beads > 65536 (the
 * scratch limit), sizes that do not match, a non-positive box, null pointers
 * or invalid excluded-volume parameters (as rpy_forces); RPY_EHIP. */
int rpy_forces_noalloc(int n_beads, int n_chains, int beads_per_chain,
                       double box_l, const double *pos, double zstar,
                       double dstar, double rcut, double *out, void *stream);

/* Synchronise the stream and report a non-finite position seen by an
 * earlier build (RPY_ENONFINITE, flag then cleared), else an adaptive order
 * that missed its tolerance at its largest order since the last call
 * (RPY_ETOL, count then cleared), else RPY_OK. */
int rpy_status(rpy_ctx *c, void *stream);

/* Orders used by the adaptive calls (bd_step, chebyshev_sqrt_apply and
 * chebyshev_sqrt_adaptive with tol > 0) settled since the last read: their
 * number, mean and largest N_Ch, and how many stopped at their largest order
 * with E_f >= tol (HOST outputs).  Synchronises the stream and resets the
 * counts. */
int rpy_order_stats(rpy_ctx *c, int64_t *calls, double *mean_order,
                    int *max_order, int64_t *missed, void *stream);

/* Copy the stored real-space part of D (FP64) into a dense row-major
 * device buffer out[3N][3N]. */
int rpy_real_space_dense(rpy_ctx *c, double *out, void *stream);

/* Per-chain observables (section "Testing and verification"):
 * re2[c] = |r_last - r_first|^2, rg2[c] = mean over beads of |r - r_cm|^2
 * (equal to the paper's pair form).  pos: device [N][3]; outputs device
 * [n_chains]. */
int rpy_observables(rpy_ctx *c, const double *pos, double *re2, double *rg2,
                    void *stream);

/* Forces used by bd_step for the given positions: out[N][3] (device).  The
 * positions are wrapped into a separate buffer, so the tables of the last
 * build (and the reciprocal sum of later products) are unaffected. */
int rpy_forces(rpy_ctx *c, const double *pos, double zstar, double dstar,
               double rcut, double *out, void *stream);

/* Gaussian noise with variance dt from Philox4x32-10 (same mapping as
 * bd_step): out[count] device. */
int rpy_gaussian_noise(double *out, int64_t count, uint64_t seed,
                       uint64_t step, double dt, void *stream);

/* Philox4x32-10 blocks: ctr_key device [n][6] uint32 (4 counter words then
 * 2 key words), out device [n][4]. */
int rpy_philox4x32_10(const uint32_t *ctr_key, uint32_t *out, int64_t n,
                      void *stream);

/* Host-only helper for tests: the 3x3 real-space block that one pair of
 * beads with wrapped separation d = r_nu - r_mu (host double[3]) receives
 * from all its images, computed by the same code the build kernel runs
 * (self = 1 adds the self term and omits the zero image).  out: host [9]. */
int rpy_host_pair_block(const rpy_params *p, const double *d, int self,
                        double *out);

/* Kernel timing for measurement.  rpy_profile_enable(c, cap) creates, once,
 * cap HIP event pairs per kernel class and from then on records a pair around
 * every launch of that class on the caller's stream (cap = 0 stops
 * recording; the events are kept until rpy_destroy).  rpy_profile_read
 * synchronises the device, returns the number of recorded launches of class
 * `kind` (RPY_PROF_*) and their summed duration in milliseconds (host
 * outputs), and resets that class.  Launches beyond cap are not recorded.
 * Packed-tile products (RPY_PROF_SYMV with stored FP64/FP32/BF16 tiles, and
 * RPY_PROF_SYMV_MULTI) have the pair recorded by their own dispatch, so it
 * times the kernel alone; the other classes take it from two stream
 * records around the launches. */
enum {
    RPY_PROF_SYMV = 0,      /* tile product of one vector (+ structure-factor
                               partials), matrix-core block product,
                               matrix-free real space */
    RPY_PROF_BUILD = 1,     /* real-space tile build */
    RPY_PROF_KSPACE = 2,    /* structure-factor reduction */
    RPY_PROF_EPI = 3,       /* reciprocal back-projection + recurrence epilogue */
    RPY_PROF_OTHER = 4,     /* bd_step's forces + noise (on an internal
                               second stream, beside the tile build) */
    RPY_PROF_SYMV_MULTI = 5, /* packed tile products of 2-4 vectors */
    RPY_PROF_KINDS = 6
};
int rpy_profile_enable(rpy_ctx *c, int cap);
int rpy_profile_read(rpy_ctx *c, int kind, int64_t *count, double *total_ms);

/* Number of wave vectors in the half-space set used per product. */
int rpy_num_kvectors(const rpy_ctx *c);

/* ------------------------------------------------------------------------
 * Batches of independent boxes (the ensembles over which section "Testing
 * and verification" averages R_e, R_g and diffusion).  Every box is its own
 * periodic system with its own N, chains, L, a, alpha and r_c; all boxes
 * must give the same integer wave-vector set (equal floor((k_c L/2 pi)^2),
 * e.g. a common alpha L and k_c/alpha).  Excluded volume is not supported
 * (theta conditions with the overlap-corrected tensor, eq. cor5).
 *
 * Layout: the beads of box b occupy the padded index range
 * [bead0[b], bead0[b] + N_b) of one global array of rpy_batch_padded_beads()
 * beads; bead0[b] is a multiple of tile_beads and the beads between boxes
 * are padding.  Every vector argument is a device FP64 array [G][3] in that
 * layout (G = padded beads), m vectors stacked with stride 3G.  Entries of
 * padding beads must be finite on input; they are zero (or untouched
 * positions) on output.
 *
 * Each stage of a call is one kernel launch over all boxes: the wrap and the
 * phase tables, the real-space tiles of every box (tile_beads beads per tile
 * side, 32 or 64; symmetric storage per box as in rpy_create), one product
 * kernel for all stored tiles plus the structure-factor partials, one
 * reduction over all boxes' wave vectors and one back-projection + epilogue.
 * ----------------------------------------------------------------------- */
typedef struct rpy_batch rpy_batch;

/* Validate every entry of p[0..nbox-1] as rpy_create does (their lowp,
 * max_rhs and cheb_keep fields are ignored) and allocate everything once.
 * lowp: RPY_PREC_F64, or RPY_PREC_F32 to also keep FP32 tiles for
 * Chebyshev products in FP32.  Errors: RPY_EINVAL (bad entry, unequal
 * wave-vector sets, tile_beads not 32/64, more than 65535 boxes, 3G beyond
 * int32), RPY_EGEOM, RPY_ENOMEM, RPY_EHIP. */
int rpy_batch_create(rpy_batch **out, const rpy_params *p, int nbox, int lowp,
                     int tile_beads);
void rpy_batch_destroy(rpy_batch *b);

/* G, the padded number of beads (-1 for NULL). */
int64_t rpy_batch_padded_beads(const rpy_batch *b);

/* bead0: host int64 [nbox + 1]; bead0[nbox] = G. */
int rpy_batch_offsets(const rpy_batch *b, int64_t *bead0);

/* Wrap pos (device [G][3]) and build the real-space tiles of every box
 * (eq. DF with the overlap form, as rpy_ewald_build per box). */
int rpy_batch_build(rpy_batch *b, const double *pos, void *stream);

/* out = D_b . v on every box for m = 1 or 2 vectors (eq. DF, full periodic
 * sum).  prec: RPY_PREC_F64, or RPY_PREC_F32 if created with FP32 tiles (the
 * reciprocal sum stays FP64). */
int rpy_batch_apply(rpy_batch *b, const double *v, double *out, int m,
                    int prec, void *stream);

/* Chebyshev approximation of sqrt(D_b) dw on every box (eq. cheb1-cheb3),
 * n_cheb terms; interval per box from the paper's rule with constant C
 * (RPY_BOUNDS_PAPER, one extra FP64 product with U+) or the explicit
 * [d_min, d_max] for all boxes.  e_f: optional device [nbox] E_f per box;
 * bounds: optional device [nbox][2] (d_min, d_max) used per box. */
int rpy_batch_chebyshev(rpy_batch *b, const double *dw, double *out,
                        int n_cheb, int bounds_rule, double C, double d_min,
                        double d_max, int prec, double *e_f, double *bounds,
                        void *stream);

/* One step of every box, as bd_step with dw = NULL: springs, D.F in FP64,
 * interval + coefficients per box, noise from Philox4x32-10 with the mapping
 * of rpy_gaussian_noise over all 3G padded entries (padding entries zero),
 * Chebyshev products in bp->prec, Euler update of the real beads.
 * bp->ev_zstar must be 0, bp->tol <= 0 (a fixed order n_cheb) and the rule
 * RPY_BOUNDS_EXPLICIT or RPY_BOUNDS_PAPER.  drift, noise: optional device [G][3]; e_f:
 * optional device [nbox]. */
int rpy_batch_step(rpy_batch *b, double *pos, const bd_params *bp,
                   uint64_t seed, uint64_t step, double *drift, double *noise,
                   double *e_f, void *stream);

/* n_steps steps with noise steps step0, step0 + 1, ...: identical to that
 * many rpy_batch_step calls, but every step is one launch of a HIP graph
 * captured from the step's kernels (captured on the first call and again
 * when pos, *bp or seed change; capture uses an internal stream).  The
 * graph holds kernel nodes only. */
int rpy_batch_run(rpy_batch *b, double *pos, const bd_params *bp,
                  uint64_t seed, uint64_t step0, int n_steps, void *stream);

/* Product variant of the batched tile kernel, for the autotuner (the values
 * are identical whichever variant runs; only the time differs):
 *   sf_place   RPY_SF_SPREAD (default): the structure-factor workgroups are
 *              spread evenly through the launch, so that their FP64
 *              arithmetic overlaps the tile stream; RPY_SF_FRONT: they are
 *              the first workgroups of the launch;
 *   tile_loads RPY_LOADS_STREAM (default): non-temporal tile loads;
 *              RPY_LOADS_CACHED: ordinary loads that allocate in the caches.
 * A change drops the captured step graph (the next rpy_batch_run captures
 * again) and synchronises the device first.  Errors: RPY_EINVAL for other
 * values. */
enum { RPY_SF_SPREAD = 0, RPY_SF_FRONT = 1 };
enum { RPY_LOADS_STREAM = 0, RPY_LOADS_CACHED = 1 };
int rpy_batch_set_variant(rpy_batch *b, int sf_place, int tile_loads);

/* Nodes (kernel launches) of the captured step graph of rpy_batch_run, or -1
 * before the first capture. */
int64_t rpy_batch_graph_nodes(const rpy_batch *b);

/* Per-chain R_e^2 and R_g^2 of all boxes, chains in box order: device
 * outputs [sum of n_chains]. */
int rpy_batch_observables(rpy_batch *b, const double *pos, double *re2,
                          double *rg2, void *stream);

/* As rpy_status, for the batch's non-finite flag. */
int rpy_batch_status(rpy_batch *b, void *stream);

/* Human-readable text for an error code (static storage). */
const char *rpy_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* RPY_H */
