/*
 * pfmp.h -- C-ABI of libpfmp, the MI355X (gfx950) hot path of polynomial-filtered
 * mass-preconditioned Hybrid Monte Carlo for two-flavour lattice QCD
 * (Haar, Kamleh, Zanotti, Nakamura, arXiv:1609.02652).
 *
 * Conventions shared by every call
 * --------------------------------
 * Return value: 0 on success, else a negative PFMP_ERR_* code; the message of
 * the last failure on a context is returned by pfmp_last_error().
 *
 * Lattice: dims[4] = (Lx, Ly, Lz, Lt), every extent even and >= 4.  Sites are
 * numbered lexicographically, lex = x + Lx*(y + Ly*(z + Lz*t)); parity =
 * (x+y+z+t) mod 2 (0 = even); the even-odd index of a site is lex/2.  Gauge links
 * are periodic; a fermion hop that crosses the t boundary takes the factor t_bc
 * (-1: antiperiodic).
 *
 * Dirac matrices: chiral basis, g_k = [[0, -i s_k], [i s_k, 0]] (k = x,y,z),
 * g_t = [[0, 1], [1, 0]], g_5 = diag(1, 1, -1, -1).  Lie algebra: T_a = lambda_a/2.
 *
 * Operators (paper Sec. 2.1 fermion matrix M, K = M^dag M; Table 3.1 "even-odd
 * Wilson", extended by the clover term):
 *   D_hop psi(x) = sum_mu [(1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^dag psi(x-mu)]
 *   M    = A - kappa D_hop,   A = 1 + i kappa c_sw sum_{mu<nu} sigma_mu_nu Fhat_mu_nu,
 *   Fhat = (Q - Q^dag)/8 over the four clover leaves, sigma = (i/2)[g_mu, g_nu],
 *   Mhat = A_ee - kappa^2 D_eo A_oo^-1 D_oe   (even sites; det M = det A_oo det Mhat),
 *   Khat = Mhat^dag Mhat  (one "K multiplication", the paper's unit of cost).
 * An operator is selected by a slot index 0..PFMP_MAX_OPS-1 configured with
 * pfmp_set_operator(); the Hasenbusch operators J = W^dag W of the paper are the
 * same operator at a heavier kappa in another slot.
 *
 * Memory: every field buffer is DEVICE memory owned by the caller (the library
 * never frees it).  Fields passed to the compute calls are in the library's
 * internal layout; pfmp_pack_* / pfmp_unpack_* convert from / to the canonical
 * layouts:
 *   gauge    [V][4][3][3] complex128 (lexicographic sites)
 *   spinor   [Vh][4][3]   complex128 on one parity (even-odd index)
 *   momenta  [V][4][8]    float64, coefficients of T_a (P = sum_a p_a T_a)
 * pfmp_field_bytes() gives the size of an internal buffer.  The context owns only
 * its geometry, gauge copy, per-slot clover fields and solver workspace.
 *
 * Ordering: every call is enqueued on the context's stream and is asynchronous,
 * except calls that return host scalars (solver statistics, actions, dot
 * products), which synchronise the stream before returning.
 */
#ifndef PFMP_H
#define PFMP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PFMP_OK 0
#define PFMP_ERR_ARG (-1)    /* null pointer, bad extent, bad slot or size */
#define PFMP_ERR_HIP (-2)    /* a HIP runtime call failed; see pfmp_last_error */
#define PFMP_ERR_NOCONV (-3) /* solver reached maxiter; x holds the last iterate */
#define PFMP_ERR_OOM (-4)    /* device allocation failed */
#define PFMP_ERR_STATE (-5)  /* call needs a gauge field / operator not yet set */

#define PFMP_MAX_OPS 8
#define PFMP_MAX_SHIFTS 128

typedef struct pfmp_ctx pfmp_ctx;

/* Precision of a field buffer or of an operator application. */
typedef enum {
    PFMP_F64 = 0,      /* complex128 storage, FP64 arithmetic */
    PFMP_F32 = 1,      /* complex64 storage, FP32 arithmetic */
    PFMP_F16 = 2       /* IEEE half spinor storage with one FP32 scale per site; FP32 arithmetic */
} pfmp_prec;

/* Kinds of internal buffers for pfmp_field_bytes. */
typedef enum {
    PFMP_FIELD_SPINOR = 0,   /* one parity */
    PFMP_FIELD_GAUGE = 1,    /* canonical gauge field (input of pfmp_set_gauge), V*4*9 complex128 */
    PFMP_FIELD_MOMENTA = 2   /* momenta / forces, V*4*8 float64 */
} pfmp_field;

/* ---- context ---------------------------------------------------------------- */

/* Create a context for a lattice.  stream: hipStream_t to enqueue on (NULL = the
 * null stream).  Errors: PFMP_ERR_ARG (odd or < 4 extent, or a volume above 2^31 - 1
 * sites), PFMP_ERR_OOM. */
int pfmp_create(const int dims[4], int t_bc, void *stream, pfmp_ctx **out);
int pfmp_destroy(pfmp_ctx *ctx);
const char *pfmp_last_error(pfmp_ctx *ctx);
/* Bytes of an internal field of the given kind and precision. */
long long pfmp_field_bytes(pfmp_ctx *ctx, int field, int prec);
/* Device kernel that writes the exact even-odd tables the stencil kernels use
 * (computed by the same device index functions): lex_of_eo[2][Vh],
 * nbr[2][Vh][8] (d = 2*mu for +mu, 2*mu+1 for -mu; even-odd index on the other
 * parity), sign[2][Vh][8] (fermion boundary factor of that hop).  Device buffers. */
int pfmp_index_maps(pfmp_ctx *ctx, int32_t *lex_of_eo, int32_t *nbr, int8_t *sign);

/* ---- fields ----------------------------------------------------------------- */

/* Upload a canonical gauge field (device buffer) into the context (synchronises
 * for the SU(3) check below).  Fields derived from the links (FP32 copy, clover
 * fields of every configured slot) are rebuilt on first use. */
int pfmp_set_gauge(pfmp_ctx *ctx, const void *U_canonical);
/* Copy the context's gauge field out in canonical layout (device buffer). */
int pfmp_get_gauge(pfmp_ctx *ctx, void *U_canonical);
/* Link row reconstruction.  pfmp_set_gauge checks every link against SU(3)
 * (|U U^dag - 1| and |det U - 1| below 1e-12); when they pass and reconstruction
 * is allowed (the default), the hopping kernels read the first two rows of each
 * link and rebuild the third as the conjugate cross product (a third fewer link
 * bytes).  The link updates keep links in SU(3).  allow = 0 turns it off; *active
 * reports whether it is in use. */
int pfmp_set_link_reconstruct(pfmp_ctx *ctx, int allow);
/* Site visit order of the operator kernels (a cache-blocking choice; results are the
 * same up to the order of floating-point sums in the block partials): zt = 0 visits the
 * sites in memory order; zt > 0 (a divisor of the z extent) visits zt z-planes of one
 * t-slice, then the same planes of the next t-slice, and so on, so that the t
 * neighbours of a group are still in L2 when they are reused. */
int pfmp_set_site_order(pfmp_ctx *ctx, int zt);
/* Streaming (non-temporal) link loads in the FP64 hopping kernels: on = 1 keeps the links,
 * read once per launch, from displacing the neighbour spinors in the caches.  The
 * default is on when the FP64 gauge field exceeds 128 MiB.  The FP32 and FP16 link copies
 * (records) are always read with cached loads. */
int pfmp_set_link_streaming(pfmp_ctx *ctx, int on);
typedef struct {
    int zt;          /* chosen site visit order (pfmp_set_site_order) */
    int stream;      /* chosen link load mode (pfmp_set_link_streaming) */
    double us_Mhat;  /* time of one FP64 Mhat application with that choice, microseconds */
} pfmp_tuning;
/* Autotuner: times one FP64 Mhat of slot op (HIP events, 10 repetitions) for every visit
 * order (0 and each divisor of the z extent from 2 to 16) with cached and with streaming
 * link loads and keeps the fastest for all later launches.  Synchronises. */
int pfmp_autotune(pfmp_ctx *ctx, int op, pfmp_tuning *out);
/* Solver iterations replayed as HIP graphs (on = 1, the default): the launches of one
 * iteration are captured once per set of buffers and operator and replayed, which takes
 * the per-launch host overhead out of the iteration.  on = 0 launches them one by one;
 * the results are the same bit for bit. */
int pfmp_set_graphs(pfmp_ctx *ctx, int on);
/* Links and clover blocks of the FP16-storage solver (prec F16): on = 1 (the default) reads
 * their FP16 copies, on = 0 the FP32 ones.  The FP16 copies move fewer bytes; on a system
 * with a harder spectrum their rounding can cost iterations (both converge to the same
 * tolerance with FP64 reliable updates).  Applies to later solves. */
int pfmp_set_half_links(pfmp_ctx *ctx, int on);
/* level 1: pfmp_trajectory and pfmp_md_evolve print one line per phase and per merged
 * step with fermion forces (solver iterations so far, seconds) to stderr; 0 (default): quiet. */
int pfmp_set_verbose(pfmp_ctx *ctx, int level);
int pfmp_get_link_reconstruct(pfmp_ctx *ctx, int *active);
/* Configure slot op with (kappa, c_sw): builds A_ee, A_oo^-1 (per-site Cholesky
 * of the two 6x6 chiral blocks) and ln det A_oo.  Needs a gauge field.  Errors:
 * PFMP_ERR_ARG (slot), PFMP_ERR_STATE (no gauge), PFMP_ERR_ARG if A_oo is not
 * positive definite. */
int pfmp_set_operator(pfmp_ctx *ctx, int op, double kappa, double csw);
/* Canonical spinor (complex128 [Vh][4][3]) <-> internal spinor of precision prec. */
int pfmp_pack_spinor(pfmp_ctx *ctx, const void *canonical, void *internal, int prec);
int pfmp_unpack_spinor(pfmp_ctx *ctx, const void *internal, void *canonical, int prec);
/* Canonical momenta / forces (float64 [V][4][8]) <-> internal. */
int pfmp_pack_momenta(pfmp_ctx *ctx, const double *canonical, double *internal);
int pfmp_unpack_momenta(pfmp_ctx *ctx, const double *internal, double *canonical);

/* ---- operators (paper Sec. 2.1; even-odd Schur form) ------------------------ */

/* out = D_eo in (out_parity 0, input odd) or D_oe in (out_parity 1, input even);
 * dagger: the blocks of D_hop^dag.  FP64. */
int pfmp_apply_hop(pfmp_ctx *ctx, int out_parity, int dagger, const void *in, void *out);
/* out = A in, or A^-1 in (inverse = 1, odd parity only), on one parity of slot op. */
int pfmp_apply_clover(pfmp_ctx *ctx, int op, int parity, int inverse, const void *in, void *out);
/* out = Mhat in (dagger 0) or Mhat^dag in = g5 Mhat g5 in (dagger 1).
 * prec PFMP_F64: FP64 fields and arithmetic; PFMP_F32: FP32 fields, links and clover.
 * PFMP_F16: in and out are FP32 fields; the input is rounded into FP16 spinor storage,
 * each stage stores its result in FP16 storage with FP32 arithmetic and the FP16 (or,
 * after pfmp_set_half_links(ctx, 0), FP32) copies of the links and clover, as the
 * FP16-storage inner solver does, and the result is widened to FP32. */
int pfmp_apply_M(pfmp_ctx *ctx, int op, int dagger, const void *in, void *out, int prec);
/* out = Khat in = Mhat^dag Mhat in; prec as for pfmp_apply_M (PFMP_F16: the intermediate
 * Mhat in is stored in FP16 as well). */
int pfmp_apply_MdagM(pfmp_ctx *ctx, int op, const void *in, void *out, int prec);

/* Khat as pfmp_apply_MdagM (prec PFMP_F64 or PFMP_F32, same kernels and bits) for callers
 * that cannot allocate device memory: code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc.  The two intermediates live in a static 128 MiB device
 * array (two spinor fields of one parity: Vh <= 349525 sites in FP64, e.g. 24^3 x 48;
 * Vh <= 699050 in FP32), which each GPU holds until the process ends; its device address
 * is looked up per GPU when a context is created.  No hipMalloc, hipFree or allocating
 * library call is made (a stale clover slot is rebuilt into its existing buffers).
 * Errors: PFMP_ERR_ARG for a lattice beyond the limit, null buffers or another precision.
 * All contexts on one GPU share the array: calls that overlap on one GPU (other streams,
 * other threads) race and must be serialised by the caller. */
int pfmp_apply_MdagM_noalloc(pfmp_ctx *ctx, int op, const void *in, void *out, int prec);

/* Product-form polynomial (paper App. A): out = norm * prod_k (Khat - z_k) in,
 * the factors applied in the order given (k = 0 first).  roots: n complex
 * numbers as 2n doubles (host); norm: complex (host).  chain: optional array of
 * n device buffers; chain[k] receives norm times the partial product after k
 * factors (chain[0] = norm * in) -- the vectors the polynomial force needs.
 * prec PFMP_F64: in, out and chain are FP64 fields; PFMP_F32: FP32 fields, the
 * operator applied with the FP32 copies of the links and clover (roots and norm
 * rounded to FP32).  out must not alias a chain buffer (PFMP_ERR_ARG). */
int pfmp_apply_poly(pfmp_ctx *ctx, int op, int n, const double *roots, const double norm[2],
                    const void *in, void *out, void *const *chain, int prec);

/* ---- solvers (paper Sec. 2.1 CG on K; App. C multi-shift) -------------------- */

typedef struct {
    double tol;          /* stop at |b - A x| <= tol |b| (relative 2-norm, recomputed in FP64 at exit) */
    int maxiter;
    int prec;            /* pfmp_prec of the inner operator; FP32/F16 use FP64 reliable updates */
    double delta;        /* reliable-update trigger: residual drop factor (mixed precision); 0 = 0.01 FP32, 0.1 FP16 */
    int check_every;     /* iterations between host convergence checks (0 = automatic) */
} pfmp_solver_params;

typedef struct {
    int iters;                  /* Krylov iterations (one Khat multiplication each) */
    int reliable_updates;
    double true_res;            /* FP64 |b - A x| / |b| of the (base) system at exit */
    double shift_res[PFMP_MAX_SHIFTS];  /* FP64 true residual per shift (multi-shift) */
    double seconds;             /* wall time of the solve */
    long long kmults;           /* Khat multiplications spent, residual checks included */
} pfmp_solver_stats;

/* CG for Khat x = b on slot op (zero initial guess).  b, x: FP64 internal spinors.
 * Returns PFMP_ERR_NOCONV (x = last iterate, stats filled) at maxiter. */
int pfmp_cg_solve(pfmp_ctx *ctx, int op, const void *b, void *x, const pfmp_solver_params *p,
                  pfmp_solver_stats *st);
/* Multi-shift CG (Jegerlehner's shifted recurrences on Hermitian positive Khat):
 * x_s = (Khat - z_s)^-1 b for nshift complex shifts z_s (2*nshift doubles, host),
 * one Khat multiplication per iteration shared by all shifts.  A zero shift is
 * allowed (it is then the base system).  FP64. */
int pfmp_cg_multishift(pfmp_ctx *ctx, int op, int nshift, const double *z, const void *b,
                       void *const *x, const pfmp_solver_params *p, pfmp_solver_stats *st);

/* ---- multi-RHS batches (several pseudofermion solves at one gauge field) ------ */

/* out_r = Khat_{ops[r]} in_r for nrhs <= 8 right-hand sides, each with its own operator
 * slot (all clover or all Wilson), each bit for bit the single-RHS Khat.  Clover batches
 * (default layout): a lane pair per site applies each leg's link, loaded once, to up to 4
 * right-hand sides (4 launches per group of 4).  Wilson batches, or after
 * pfmp_set_batch_layout(ctx, 0): one workgroup per (site block, rhs), the workgroups of one
 * site block adjacent so that they share the links through L2 (4 launches).  prec
 * PFMP_F64 or PFMP_F32 internal spinors (FP32: FP32 links and clover). */
int pfmp_apply_MdagM_batch(pfmp_ctx *ctx, int nrhs, const int *ops, const void *const *in, void *const *out,
                           int prec);
/* layout of the batched clover stencils (apply and CG): 1 (default) the default group of rhs
 * per lane pair sharing each link load (4); 2 or 4 groups of that many rhs per lane pair;
 * 0 one workgroup per (site block, rhs).  Same results in every layout.  Other values:
 * PFMP_ERR_ARG. */
int pfmp_set_batch_layout(pfmp_ctx *ctx, int multi);
/* CG for Khat_{ops[r]} x_r = b_r, r < nrhs <= 8, all iterated in the same launches;
 * a converged right-hand side stops.  b, x: FP64 internal spinors; st: nrhs records.
 * p->prec PFMP_F64: CG in FP64.  PFMP_F32 (and PFMP_F16, taken as FP32): defect
 * correction, FP64 residuals and solution around batched FP32 CG passes (FP32 links and
 * clover), each to a relative 2e-6 or what the remaining reduction needs;
 * st->reliable_updates counts the passes, st->iters the FP32 iterations.  Every
 * right-hand side stops on its FP64 true residual <= tol |b_r|. */
int pfmp_cg_solve_batch(pfmp_ctx *ctx, int nrhs, const int *ops, const void *const *b, void *const *x,
                        const pfmp_solver_params *p, pfmp_solver_stats *st);

/* ---- learned preconditioner and flexible CG ------------------------------------ */

/* Gauge-covariant parallel-transport convolution network N (2 layers, 4 -> 12 -> 4
 * complex colour-vector channels, norm gate h/(1+|h|^2), skip term W0): weights W are
 * 784 complex numbers (1568 doubles, host) laid out [W1 8x12x4 | W2 8x4x12 | W0 4x4];
 * FP32 weights and arithmetic.  out = N(r) = |r| z(r/|r|) (FP64 internal spinors). */
int pfmp_ptnet_apply(pfmp_ctx *ctx, const double *W, const void *r, void *out);
/* Training loss over n training vectors r_p and its gradient matrices A (1568 doubles,
 * host, same layout as W) with dLoss = 2 Re sum A dW.  Two objectives:
 *   op >= 0 (preconditioned residual, on slot op's Khat in FP32):
 *           sum_p |Khat z(rhat_p) - rhat_p|^2,  rhat_p = r_p / |r_p|;  e may be NULL;
 *   op <  0 (solution matching, pairs with Khat e_p = r_p):
 *           sum_p |z(rhat_p) - e_p/|r_p||^2 / |e_p/|r_p||^2. */
int pfmp_ptnet_grad(pfmp_ctx *ctx, const double *W, int op, int n, const void *const *r, const void *const *e,
                    double *loss, double *A);
/* Adam (beta 0.9, 0.999) on the real and imaginary parts of W for `steps` full-batch
 * steps of pfmp_ptnet_grad's objective (op as there); W (1568 doubles, host) updated in
 * place; losses[steps] optional. */
int pfmp_ptnet_train(pfmp_ctx *ctx, double *W, int op, int n, const void *const *r, const void *const *e,
                     int steps, double lr, double *losses);
/* Flexible CG on Khat (Notay 2000 with one direction kept, Polak-Ribiere beta) with N as
 * preconditioner; W = NULL uses the identity (then it is CG).  Plain CG is the fallback:
 * a step whose <N(r), r> <= 0 takes z = r, and when |r| has not halved within 100
 * iterations the rest of the solve is plain CG from the current iterate.  Stops on the
 * FP64 true residual |b - Khat x| <= tol |b|, like pfmp_cg_solve; stats->reliable_updates
 * counts the plain-CG steps. */
int pfmp_fcg_solve(pfmp_ctx *ctx, int op, const double *W, const void *b, void *x, const pfmp_solver_params *p,
                   pfmp_solver_stats *st);
/* CG on Khat that copies (x_k, r_k) at the iterations snap_iters (ascending) into the
 * caller's buffers; training pairs are then (r_k, x - x_k).  *ntaken = snapshots made. */
int pfmp_cg_harvest(pfmp_ctx *ctx, int op, const void *b, void *x, double tol, int maxiter, int nsnap,
                    const int *snap_iters, void *const *snap_x, void *const *snap_r, int *ntaken);

/* ---- BLAS-1 on internal FP64 spinors (FP64 reductions, deterministic order) -- */

/* *out = <a, b> (complex, 2 doubles on the host). */
int pfmp_dot(pfmp_ctx *ctx, const void *a, const void *b, double out[2]);
/* y = alpha x + beta y (complex alpha, beta). */
int pfmp_axpby(pfmp_ctx *ctx, const double alpha[2], const void *x, const double beta[2], void *y);
/* out = in converted between the internal FP64 and FP32 spinor fields of one parity
 * (prec_in, prec_out each PFMP_F64 or PFMP_F32; round to nearest into FP32).  in and
 * out must not overlap unless prec_in == prec_out, which copies. */
int pfmp_convert_spinor(pfmp_ctx *ctx, const void *in, int prec_in, void *out, int prec_out);

/* ---- forces (paper App. C) and integrator updates (App. B) ------------------ */

/* F += sum_p d/dw Re[ c_p X_p^dag Mhat_op Y_p ] along U_mu(x) -> exp(i w T_a) U_mu(x),
 * for npairs pairs of FP64 internal spinors X_p, Y_p (device) with complex
 * coefficients c_p (2*npairs doubles, host).  flags: PFMP_FORCE_HOP and/or
 * PFMP_FORCE_CLOVER select the parts of dMhat (neither = the full derivative);
 * PFMP_FORCE_F32: X_p, Y_p are FP32 internal spinors, their odd-site
 * intermediates are formed by the FP32 operator and the force is summed in FP64.
 * F: internal momenta layout, accumulated. */
#define PFMP_FORCE_HOP 1
#define PFMP_FORCE_CLOVER 2
#define PFMP_FORCE_F32 4
int pfmp_fermion_force(pfmp_ctx *ctx, int op, int npairs, const void *const *X, const void *const *Y,
                       const double *coeff, int flags, double *F);
/* F += coef * d/dw S_det, S_det = -2 sum_{x odd} ln det A(x) of slot op. */
int pfmp_logdet_force(pfmp_ctx *ctx, int op, double coef, double *F);
/* F += d/dw S_G, Wilson gauge action S_G = beta sum_P (1 - Re tr U_P / 3). */
int pfmp_gauge_force(pfmp_ctx *ctx, double beta, double *F);
/* S[eps]: P <- P - eps F (internal momenta layout). */
int pfmp_update_momenta(pfmp_ctx *ctx, double eps, const double *F, double *P);
/* T[eps]: U_mu(x) <- exp(i eps P_mu(x)) U_mu(x); rebuilds every configured operator. */
int pfmp_update_gauge(pfmp_ctx *ctx, double eps, const double *P);

/* ---- actions (FP64, host results) ------------------------------------------ */

/* S_G of the context's gauge field. */
int pfmp_gauge_action(pfmp_ctx *ctx, double beta, double *out);
/* -2 sum_{x odd} ln det A(x) of slot op. */
int pfmp_logdet_action(pfmp_ctx *ctx, int op, double *out);
/* sum over links of tr P^2 (internal momenta). */
int pfmp_kinetic(pfmp_ctx *ctx, const double *P, double *out);

/* ---- PF-MP HMC (paper Sec. 2.1, eq. pfmp_action, App. B, App. C) ------------ */

/* Filter terms of the action.  J = W^dag W is the operator of slot `op` (a
 * heavier kappa); K_b is the operator of slot `op2`. */
typedef enum {
    PFMP_TERM_POLY = 0,      /* phi^dag P(J) phi, P the degree-n Chebyshev filter of App. A        */
    PFMP_TERM_POLYCORR = 1,  /* phi^dag [J P(J)]^-1 phi (pole sum + multi-shift CG, App. C)         */
    PFMP_TERM_RATIO = 2,     /* phi^dag W^dag K_b^-1 W phi: the Hasenbusch ratio J K_b^-1            */
    PFMP_TERM_HEAVY = 3,     /* phi^dag J^-1 phi                                                  */
    PFMP_TERM_POLYQ = 4      /* phi^dag Q(J) phi, Q = P_n / P_n1: the intermediate filter of the
                                2-filter actions (eq. 2poly); P_n1 divides P_n when (n1 + 1)
                                divides (n + 1) (App. A), and Q has the n - n1 roots of P_n that
                                are not roots of P_n1, norm a_n / a_n1                            */
} pfmp_term_kind;

#define PFMP_MAX_TERMS 16

typedef struct {
    int kind;        /* pfmp_term_kind */
    int op;          /* slot of J (W) */
    int op2;         /* RATIO: slot of the denominator K_b */
    int n;           /* POLY / POLYCORR: polynomial degree (even) */
    double mu, nu;   /* Chebyshev ellipse (mu >= nu > 0) */
    int steps;       /* 2MN steps of this term over the trajectory */
    int n1;          /* POLYQ: degree of the inner filter P_n1 (even, (n1 + 1) | (n + 1)) */
} pfmp_term;

typedef struct {
    double beta;          /* Wilson gauge coupling */
    int det_op;           /* slot whose -2 ln det A_oo enters the action (-1: none) */
    int gauge_steps;      /* 2MN steps of the gauge scale (and of S_det when det_steps is 0) */
    double tau;           /* trajectory length */
    double lambda;        /* 2MN parameter; 0 selects 0.1931833275037836 (minimum norm) */
    int nterms;
    const pfmp_term *terms;
    double tol;           /* relative residual of every solve */
    int maxiter;
    int exact_start;      /* 1: evaluate the filter actions at the start; 0: use eta^dag eta */
    int solver_prec;      /* pfmp_prec of the CG solves (RATIO, HEAVY): F32 / F16 use FP64 reliable updates */
    const double *ptnet;  /* optional learned-preconditioner weights (1568 doubles): the CG solves become
                             flexible CG with that network; NULL: plain CG */
    int batch;            /* 1: the CG solves of all RATIO / HEAVY terms due at the same merged step run
                             as one multi-RHS solve (the S_j commute, App. B), with the correction
                             term's z = 0 pole in the FP32 / F16 modes; FP64, or FP32 passes inside
                             FP64 defect correction in those modes; not with ptnet */
    int det_steps;        /* > 0: S_det on its own 2MN scale with this many steps (one more row of the
                             merged schedule); 0: S_det moves with the gauge action */
} pfmp_hmc_spec;

typedef struct {
    double H0, H1, dH;
    int accept;
    int nsteps;                          /* length of the merged schedule */
    int nforce[PFMP_MAX_TERMS + 1];      /* force evaluations: [0] gauge (+S_det), [1+j] term j */
    long long kmults;                    /* Khat / J multiplications, the paper's N_mat unit */
    long long solver_iters;
    double seconds;
    double parts0[PFMP_MAX_TERMS + 3];   /* kinetic, S_G, S_det, terms at the start */
    double parts1[PFMP_MAX_TERMS + 3];   /* ... at the end */
    int nforce_det;                      /* S_det force evaluations on its own scale (det_steps > 0) */
} pfmp_traj_stats;

/* Pseudofermion heatbath: phi_j with density exp(-S_j) from Gaussian eta_j
 * (density exp(-eta^dag eta)); device FP64 internal spinors, one per term. */
int pfmp_heatbath(pfmp_ctx *ctx, const pfmp_hmc_spec *spec, const void *const *eta, void *const *phi);
/* H = sum tr P^2 + S_G + S_det + sum_j S_j(phi_j); parts (nterms + 3 doubles) optional. */
int pfmp_hamiltonian(pfmp_ctx *ctx, const pfmp_hmc_spec *spec, const double *P, const void *const *phi,
                     double *H, double *parts);
/* Force sizes for step-size tuning (Sec. 2.4: F_i h_i = const with the maximal force):
 * each row's force at the context's gauge field with pseudofermions phi, as the norm
 * (sum_a F_a^2)^(1/2) of its 8 coefficients per link; out (2 (nterms + 2) doubles, host)
 * holds (maximum over links, mean over links) for the gauge action, each term in order,
 * then S_det (zeros when det_op < 0).  Terms use the spec's solver precision.  Synchronises. */
int pfmp_force_norms(pfmp_ctx *ctx, const pfmp_hmc_spec *spec, const void *const *phi, double *out);
/* Molecular dynamics over tau: the per-term 2MN schemes merged by the generalized
 * multi-scale scheme (App. B); T[eps] then the S_j of the merged step.  P
 * (internal momenta) and the context's gauge field are updated in place. */
int pfmp_md_evolve(pfmp_ctx *ctx, const pfmp_hmc_spec *spec, double *P, const void *const *phi,
                   pfmp_traj_stats *st);
/* One trajectory from the context's gauge field: heatbath, H0, MD, H1, Metropolis
 * with the uniform u (accept iff u < exp(-dH)); on reject the start field is
 * restored.  P0 is not modified; P_end (optional) receives the final momenta.
 * Errors: when any step fails (PFMP_ERR_NOCONV from a solve that reached maxiter,
 * PFMP_ERR_OOM, PFMP_ERR_HIP) the context's gauge field is also restored to the start
 * field (derived clover fields are rebuilt on next use) and the code of the failure is
 * returned, with its text in pfmp_last_error; P_end and st are then undefined. */
int pfmp_trajectory(pfmp_ctx *ctx, const pfmp_hmc_spec *spec, const double *P0, const void *const *eta, double u,
                    double *P_end, pfmp_traj_stats *st);

/* ---- host-only helpers ------------------------------------------------------ */

/* Chebyshev roots z_k = mu(1 - cos th_k) - i sqrt(mu^2-nu^2) sin th_k,
 * th_k = 2 pi k/(n+1), k = 1..n, and a_n = 1/(mu prod (mu - z_k)) (paper App. A).
 * roots: 2n doubles; norm: 2 doubles. */
int pfmp_chebyshev(int n, double mu, double nu, double *roots, double norm[2]);
/* Generalized multi-scale merge (paper App. B): nterms schemes given as integer
 * tick lists T_j (time steps, first entry 0) and S_j (space steps, any values),
 * lengths len[j], flattened one after another.  All T_j must sum to the same
 * total.  Writes the merged T' (ticks) and S'_j (nterms x nout, row-major) and
 * *nout.  cap = capacity of T_out (S_out holds nterms*cap).  PFMP_ERR_ARG on
 * unequal totals or too small a capacity. */
int pfmp_schedule_build(int nterms, const int *len, const int64_t *T_ticks, const double *S_steps,
                        int cap, int64_t *T_out, double *S_out, int *nout);

#ifdef __cplusplus
}
#endif
#endif
