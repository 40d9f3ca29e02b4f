/*
 * nep.h -- C ABI of the MI355X contour-integral moment library (libnep).
 *
 * Problem statement.  A nonlinear eigenvalue problem T(lambda) x = 0 is given
 * in split form T(z) = sum_{i=1..ell} A_i f_i(z) (Campos & Roman, Section 2,
 * eq. (split)), with constant n x n matrices A_i and scalar functions f_i
 * described with the semantics of the paper's FN object (Section 3.2.2).
 *
 * The library computes, for a closed contour Gamma (a circle or an ellipse,
 * the RG regions of Section 3.2.4), the moments
 *
 *     S_p = sum_j w_j zeta_j^p T(z_j)^{-1} V ,   p = 0 .. 2K-1,
 *
 * a trapezoid discretization of (1/(2 pi i)) oint phi(z)^p T(z)^{-1} V dz with
 * phi(z) = (z-c)/rho.  By Keldysh's expansion of the resolvent (Section 2,
 * eq. (resolvent)) only the eigenvalues inside Gamma contribute.  From the
 * block-Hankel matrices of the moments it extracts a minimal invariant pair
 * (Section 2, eqs. (invpair), (invpair-split)): the eigenvalues inside Gamma
 * and their eigenvectors, with the backward error of eq. (sressplit) in
 * infinity norms (Section 6).
 *
 * Conventions common to every call.
 *   - Every call returns a nep_status: 0 (NEP_OK) or a negative error code.
 *     No call aborts the process.  nep_last_error() returns a thread-local
 *     message describing the last failure on the calling thread.
 *   - Complex numbers are interleaved (re, im) pairs of doubles, compatible
 *     with C99 double _Complex and with numpy complex128.
 *   - Matrices passed in are column-major with a leading dimension.
 *   - "device" pointers are HIP device memory on the current device (for
 *     example the data_ptr() of a PyTorch tensor); "host" pointers are
 *     ordinary process memory.  The library never frees caller memory.
 *   - Streams are hipStream_t values passed as void*; NULL is the default
 *     stream.
 *   - Handles are not thread-safe: calls that use the same handle must not
 *     overlap.  Distinct handles may be used concurrently on distinct
 *     streams.
 */
#ifndef NEP_H
#define NEP_H

#ifdef __cplusplus
extern "C" {
#endif

typedef int nep_status;

enum {
  NEP_OK = 0,
  NEP_ERR_ARG = -1,             /* invalid argument (message says which)        */
  NEP_ERR_OOM = -2,             /* device or host allocation failed             */
  NEP_ERR_SINGULAR = -3,        /* exact zero pivot in T(z_j); node in stats    */
  NEP_ERR_NOT_HOLOMORPHIC = -4, /* a node lies on a pole or branch cut of f_i   */
  NEP_ERR_REFINE = -5,          /* refinement did not converge, fallback off    */
  NEP_ERR_RANK = -6,            /* moment rank == K*L: increase L or K          */
  NEP_ERR_DEVICE = -7,          /* HIP runtime error                            */
  NEP_ERR_BUSY = -8             /* server: no slot or memory for the query now  */
};

/* ------------------------------------------------------------------------ */
/* Scalar functions (FN semantics, Section 3.2.2)                            */
/* ------------------------------------------------------------------------ */

typedef enum {
  NEP_FN_RATIONAL = 0, /* p(x)/q(x), coefficient lists highest degree first     */
  NEP_FN_EXP = 1,      /* e^x                                                    */
  NEP_FN_LOG = 2,      /* principal log, cut on (-inf, 0]                        */
  NEP_FN_SQRT = 3,     /* principal square root, cut on (-inf, 0]                */
  NEP_FN_INVSQRT = 4,  /* 1/sqrt(x), principal branch                            */
  NEP_FN_PHI = 5,      /* phi_k: phi_0 = e^x, phi_k = (phi_{k-1} - 1/(k-1)!)/x   */
  NEP_FN_COMBINE = 6   /* two functions combined by comb_op                      */
} nep_fn_type;

typedef enum {
  NEP_COMB_ADD = 0,    /* a(x) + b(x)                                            */
  NEP_COMB_MUL = 1,    /* a(x) * b(x)                                            */
  NEP_COMB_DIV = 2,    /* a(x) / b(x)                                            */
  NEP_COMB_COMPOSE = 3 /* b(a(x)): a is applied first                            */
} nep_comb_op;

/* f(z) = beta * g(alpha * z)  (the argument and result scaling of FNSetScale).
 * Coefficient arrays, phi_k and the combine children are read during
 * nep_split_create and copied; the caller may free them afterwards.
 * A tree may hold at most 64 nodes and rational degrees at most 32. */
typedef struct nep_fn {
  int type;                      /* nep_fn_type                                  */
  double alpha[2];               /* complex argument scale (1,0 for none)        */
  double beta[2];                /* complex result scale (1,0 for none)          */
  int nnum, nden;                /* RATIONAL: coefficient counts (nden may be 0) */
  const double* num;             /* RATIONAL: host, nnum complex, highest first  */
  const double* den;             /* RATIONAL: host, nden complex, highest first  */
  int phi_k;                     /* PHI: k >= 0                                  */
  int comb_op;                   /* COMBINE: nep_comb_op                         */
  const struct nep_fn* comb_a;   /* COMBINE: first operand (host)                */
  const struct nep_fn* comb_b;   /* COMBINE: second operand (host)               */
} nep_fn;

/* ------------------------------------------------------------------------ */
/* Split operator handle (NEPSetSplitOperator, Section 3.2.2)                */
/* ------------------------------------------------------------------------ */

typedef enum {
  NEP_MAT_REAL_F64 = 0,    /* real double, column-major                          */
  NEP_MAT_COMPLEX_F64 = 1  /* complex double (interleaved), column-major         */
} nep_mat_type;

typedef struct {
  int type;                /* nep_mat_type                                        */
  const void* data;        /* n x n column-major matrix, leading dimension ld     */
  long long ld;            /* >= n, in elements                                   */
  int on_device;           /* 0: host pointer, 1: device pointer                  */
} nep_mat;

typedef struct nep_split_s* nep_split;

/* Creates a handle for T(z) = sum_i f_i(z) A_i.
 *   n      : matrix size, 1 <= n <= 4096.
 *   ell    : number of terms, 1 <= ell <= 16.
 *   A      : host array of ell matrix descriptors; the data are copied to the
 *            device (stored row-major there) before the call returns.
 *   f      : host array of ell function descriptors (copied).
 *   stream : stream used by every call on this handle (NULL = default).
 *   out    : receives the handle.
 * Errors: NEP_ERR_ARG for bad sizes or descriptors, NEP_ERR_OOM,
 * NEP_ERR_DEVICE. */
nep_status nep_split_create(int n, int ell, const nep_mat* A, const nep_fn* f,
                            void* stream, nep_split* out);

/* Frees the handle, its device copies of A_i and its resident workspace
 * (factors, solves), and sets *h = NULL (NEPDestroy(&nep) style). */
nep_status nep_split_destroy(nep_split* h);

/* Size n and term count ell of a handle. */
nep_status nep_split_info(nep_split h, int* n, int* ell);

/* ------------------------------------------------------------------------ */
/* Moments                                                                   */
/* ------------------------------------------------------------------------ */

/* Contour (RG region, Section 3.2.4).
 *   kind 0: circle  z = c + rho e^{i theta}
 *   kind 1: ellipse z = c + rho (cos theta + i v sin theta), v > 0
 * Nodes sit at theta_j = 2 pi (j + 1/2)/N (counter-clockwise); weights
 * w_j = rho (v cos theta_j + i sin theta_j)/N (v = 1 for a circle). */
typedef struct {
  int kind;
  double c[2];   /* complex centre                                            */
  double rho;    /* radius / horizontal semi-axis, > 0                        */
  double v;      /* ellipse: vertical/horizontal semi-axis ratio, > 0         */
} nep_contour;

typedef enum {
  NEP_PREC_FP64 = 0,     /* plain: complex FP64 assembly, LU (FP64 MFMA), solve */
  NEP_PREC_C32_IR64 = 1  /* mixed: complex FP32 LU and solves on FP32 MFMA with
                            FP64 residuals, corrections and moments             */
} nep_precision;

typedef struct {
  int N;             /* quadrature nodes, 2 <= N <= 1024                        */
  int L;             /* probe columns, 1 <= L <= 64                             */
  int K;             /* Hankel block rows; moments p = 0..2K-1; 2K-1 <= N-1     */
  int prec;          /* nep_precision                                          */
  int max_refine;    /* refinement sweeps (mixed); 0..20, default 5             */
  int fp64_fallback; /* 1: nodes whose refinement stalls are re-solved in FP64  */
  double refine_tol; /* stop when ||R||_inf <= tol (||T||_inf ||Y||_inf + ||V||_inf)
                        per probe column; 0 selects 1e-15                     */
  void* stream;      /* NULL: the handle's stream                               */
} nep_ciss_opts;

typedef struct {
  int N;                  /* nodes processed                                     */
  int refine_sweeps;      /* sweeps run (max over nodes)                         */
  int n_fallback;         /* nodes re-solved in FP64                             */
  int n_unconverged;      /* nodes not meeting refine_tol after all sweeps       */
  int singular_node;      /* first node with an exact zero pivot, or -1          */
  int bad_node;           /* first node on a pole/branch cut, or -1              */
  double max_rel_residual;/* max over nodes/columns of the final scaled residual */
  float ms_total;         /* device time of the call (events), if synchronous    */
  float ms_lu;            /* device time from the first LU launch to the end of
                             the factorizations (events; single calls and eager
                             batch runs; 0 for graph replays)                    */
  double min_abs_pivot;   /* smallest |u_kk| over the node factorizations in the
                             path's precision (complex FP32 for the mixed path);
                             0 with NEP_ERR_SINGULAR, NaN if a factor holds NaN  */
} nep_ciss_stats;

/* S_p = sum_j w_j zeta_j^p T(z_j)^{-1} V for p = 0..2K-1.
 *   V : device, complex n x L, column-major (ld = n), caller-owned.
 *   S : device, complex n x L x 2K, column-major; block p (n x L) starts at
 *       S + p*n*L complex entries.  Overwritten.
 *   st: if non-NULL the call waits for the stream, fills *st and returns
 *       device-detected errors (NEP_ERR_SINGULAR, NEP_ERR_NOT_HOLOMORPHIC,
 *       NEP_ERR_REFINE).  If NULL the call returns after enqueueing the work;
 *       device-detected errors are then returned by nep_ciss_wait.
 * The factors of T(z_j) stay resident in the handle until the next call with
 * different (N, prec) or until destroy. */
nep_status nep_ciss_moments(nep_split h, const nep_contour* g,
                            const nep_ciss_opts* o, const void* V, void* S,
                            nep_ciss_stats* st);

/* Waits for the last nep_ciss_moments on h and reports its status/stats. */
nep_status nep_ciss_wait(nep_split h, nep_ciss_stats* st);

/* Moments of further probes on the factors resident from the last
 * nep_ciss_moments call on h (same contour, N, L, K and precision; no
 * assembly and no factorization): solves, refinement and moments only.
 *   V: device, complex n x L (the last call's L), column-major.
 *   S: device; moment p (n x L column-major) is written at S + p*s_stride
 *      complex entries (s_stride 0: n*L).  A stride of n*L_total with S
 *      offset by j*n*L places the block as columns j*L.. of moments with
 *      L_total columns, for probe augmentation.
 *   st as in nep_ciss_moments (non-NULL: synchronous).
 * Errors: NEP_ERR_ARG if there are no resident factors or a call is still
 * pending; otherwise as nep_ciss_moments. */
nep_status nep_ciss_moments_more(nep_split h, const void* V, void* S,
                                 long long s_stride, nep_ciss_stats* st);

/* Number of eigenvalues inside the contour by the argument principle:
 * eigenvalues are the zeros of det T(z) (Section 2, eq. (nep)), so the
 * count is the winding number of det T along the contour, read from the LU
 * factors at the nodes (det T(z_j) = sign(P) prod_k u_kk) as the sum of the
 * phase steps between consecutive nodes, each taken in (-pi, pi].  It is
 * exact when det T turns by less than pi between neighbouring nodes:
 * *max_step (radians) reports the largest step, *winding the unrounded sum
 * over 2 pi.
 *   nep_ciss_count: from the factors resident from the last nep_ciss_moments
 *   call on h (its N quadrature nodes; no further factorization).
 *   nep_count_eigs: factors T at N nodes of g itself (4 <= N <= 4096) in the
 *   given precision, without solves (use N well above the count).
 * Errors: NEP_ERR_NOT_HOLOMORPHIC (a node on a pole or cut),
 * NEP_ERR_SINGULAR (det T(z_j) zero in the factor precision). */
nep_status nep_ciss_count(nep_split h, int* count, double* max_step, double* winding);
nep_status nep_count_eigs(nep_split h, const nep_contour* g, int N, int prec,
                          int* count, double* max_step, double* winding);

/* ------------------------------------------------------------------------ */
/* Extraction (minimal invariant pair, Section 2)                            */
/* ------------------------------------------------------------------------ */

typedef struct {
  double rank_tol;  /* keep singular values > rank_tol * sigma_1; 0 -> 1e-12    */
  double eta_tol;   /* convergence tolerance on the backward error eta of
                       eq. (sressplit) (the paper's NEPSetTolerances tol, Table 1
                       uses 1e-8 for most problems); 0 -> 1e-8                  */
  int max_eigs;     /* capacity of the output arrays (>= 1)                     */
  int polish_its;   /* 0: off.  > 0: pairs inside the contour whose eta exceeds
                       eta_tol are polished by residual inverse iteration (as
                       nep_rii_polish, tol 1e-14) with at most polish_its outer
                       steps before they are flagged                          */
} nep_extract_opts;

/* From S (as written by nep_ciss_moments with the same g and o) computes the
 * eigenpairs of the minimal invariant pair carried by the moments.
 *   m      : host, number of eigenpairs returned (= the numerical rank).
 *   lambda : host, 2*max_eigs doubles: complex eigenvalues, sorted by
 *            (Re, Im).
 *   X      : device, complex n x max_eigs column-major: eigenvectors,
 *            ||x||_2 = 1, largest-modulus entry real positive.
 *   eta    : host, max_eigs doubles: backward error eq. (sressplit), inf-norms.
 *   inside : host, max_eigs ints: 1 if the eigenvalue lies inside the contour
 *            and the pair has converged (eta <= eta_tol); 2 if it lies inside
 *            but eta > eta_tol (not converged: a spurious pair from a rank
 *            taken at the moments' noise floor, or one limited by the
 *            quadrature); 0 if it lies outside (the region filter of
 *            Section 3.2.4).
 *   sigma  : host, optional (may be NULL), K*L doubles: singular values of the
 *            block-Hankel matrix B0.
 * Synchronous.  NEP_ERR_RANK if every one of the K*L singular values is
 * significant (the contour holds more eigenvalues than K*L can resolve);
 * NEP_ERR_ARG if the rank exceeds max_eigs. */
nep_status nep_extract(nep_split h, const nep_contour* g, const nep_ciss_opts* o,
                       const void* S, const nep_extract_opts* e, int* m,
                       double* lambda, void* X, double* eta, int* inside,
                       double* sigma);

/* Eigenvalues inside the contour end to end, with probe augmentation:
 * moments with the first L = o->L columns of V, extraction, and while the
 * moments' rank saturates (NEP_ERR_RANK with every one of the K*L singular
 * values significant) the next L columns are solved on the resident factors
 * (nep_ciss_moments_more) and the extraction is repeated on the moments of
 * all probes so far, up to Lmax columns.
 *   V: device, complex n x Lmax column-major (the probe pool; Lmax a
 *      multiple of L, <= 256).  Outputs as nep_extract, with sigma holding
 *      K*Lmax doubles; *L_used: probe columns in the final moments; st: the
 *      first moments call's stats (optional).
 * Returns nep_extract's status for the last extraction. */
nep_status nep_eigs(nep_split h, const nep_contour* g, const nep_ciss_opts* o,
                    const nep_extract_opts* e, const void* V, int Lmax, int* m,
                    double* lambda, void* X, double* eta, int* inside,
                    double* sigma, int* L_used, nep_ciss_stats* st);

/* ------------------------------------------------------------------------ */
/* Left eigenvectors and the resolvent (Section 2, eqs. (nep-left),          */
/* (resolvent); Section 3.2.5)                                               */
/* ------------------------------------------------------------------------ */

/* Handle of the adjoint operator T^*(z) = T(conj z)^* = sum_i conj(f_i(conj z))
 * A_i^* (conjugate-transposed matrices; functions with conjugated
 * coefficients and scales).  Its right eigenpairs (y, conj(lambda)) are the
 * left eigenpairs of T: "left eigenvectors can be computed as right
 * eigenvectors of T^*" (Section 2).  Every call of this header applies to it;
 * run the moments with the conjugated contour (centre conj(c)).  Destroy
 * with nep_split_destroy. */
nep_status nep_split_adjoint(nep_split h, nep_split* out);

/* Left eigenvectors y^* T(lambda) = 0 for m given eigenvalues, by residual
 * inverse iteration on T^* with the target conj(lambda) (as nep_rii_polish on
 * the adjoint, made and kept inside h on first use).
 *   lambda: host 2m doubles (in: the eigenvalues; out: refined from the
 *           left problem), Y: device complex n x m column-major (in: start
 *           vectors, e.g. random; out: ||y||_2 = 1, largest-modulus entry
 *           real positive), eta: host m doubles (out): backward errors of
 *           (y, conj(lambda)) for T^* (eq. (sressplit), inf-norms of A_i^*).
 *   max_it: 1..100 outer steps. */
nep_status nep_left_eigenvectors(nep_split h, int m, double* lambda, void* Y,
                                 double* eta, int max_it);

/* Action of the resolvent's eigen-part on L vectors (NEPApplyResolvent):
 *   W = sum_q (z - lambda_q)^{-1} x_q y_q^* V / (y_q^* T'(lambda_q) x_q),
 * Keldysh's expansion (eq. (resolvent)) without its holomorphic remainder
 * R(z), with the normalization y^* T'(lambda) x = 1 applied explicitly (so x
 * and y may have any scaling).  Exact for T^{-1}(z) when the pairs are all
 * of T's (semisimple) eigenvalues and R = 0, e.g. a linear T with every
 * eigenvalue given.
 *   lambda: host 2m doubles; X, Y: device complex n x m (right and left
 *   eigenvectors); z: host complex (2 doubles), not an eigenvalue;
 *   V: device complex n x L; W: device complex n x L (out).
 * Errors: NEP_ERR_ARG if some y^* T'(lambda) x = 0 (not a simple
 * eigenvalue). */
nep_status nep_apply_resolvent(nep_split h, int m, const double* lambda,
                               const void* X, const void* Y, const double* z,
                               int L, const void* V, void* W);

/* T(z_k)^{-1} V at m points z_k (host, 2m doubles): the full resolvent,
 * by assembly, LU and solves in the given precision (the mixed path refines
 * in FP64 as the moments do).  V: device complex n x L (L <= 64);
 * Y: device, m blocks of n x L column-major (block k at Y + k*n*L).
 * st: optional stats (synchronous either way). */
nep_status nep_solve_at(nep_split h, int m, const double* z, int L,
                        const void* V, int prec, void* Y, nep_ciss_stats* st);

/* Backward errors eq. (sressplit) (inf-norms) of m given pairs.
 *   lambda: host, m complex; X: device, complex n x m column-major;
 *   eta: host, m doubles. */
nep_status nep_backward_error(nep_split h, int m, const double* lambda,
                              const void* X, double* eta);

/* FP64 polish of m eigenpairs by residual inverse iteration (Section 4.1,
 * Algorithm "RII", eqs. (rii), (rii-scalar)), all pairs at once.  For each
 * pair the target sigma is its own eigenvalue; T(sigma) is assembled and
 * factored in complex FP64 on the device once, and each outer step solves the
 * scalar equation x^* T(sigma)^{-1} T(z) x = 0 by Newton's method with the
 * FN derivatives (FNEvaluateDerivative, Section 3.2.2) to |mu|/|z| <
 * sqrt(eps), stops when eta(x, lambda) < tol (eq. (sressplit), infinity
 * norms), and otherwise corrects x <- (x - T(sigma)^{-1} r)/||.||, r = T(lambda) x.
 *   lambda: host, 2m doubles (in/out); X: device, complex n x m column-major
 *   (in/out; returned with ||x||_2 = 1 and the largest-modulus entry real
 *   positive); eta: host, m doubles (out): the pairs' backward errors after
 *   the call.  A pair is replaced only if its backward error decreased.
 *   tol: 0 selects 1e-14.  max_it: 1..100 outer steps.
 *   iters: host, m ints (optional): outer steps each pair took (0: left as
 *   it was, e.g. sigma an eigenvalue to working precision).
 * Synchronous, on the handle's stream.  Allocates device memory (factors of
 * m matrices of size n in complex FP64). */
nep_status nep_rii_polish(nep_split h, int m, double* lambda, void* X,
                          double* eta, double tol, int max_it, int* iters);

/* nep_backward_error for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same computation and results, with every device buffer it
 * needs (function values, the n x m residual block, column maxima, term
 * tables) in one library-owned scratch array of 4.125 MiB per GPU, held from
 * the first call on that GPU until the process ends.  It calls no hipMalloc,
 * hipFree or other allocating routine.
 *   Limits: m <= 256 and n*m <= 262144; larger requests return NEP_ERR_ARG
 *   before any device work.
 *   Every call on a GPU uses that GPU's one scratch array, so calls that
 *   overlap on one GPU (from several host threads, or on several streams
 *   before the earlier call returned) race; calls are synchronous and each
 *   overwrites everything it reads, so sequential calls are independent.
 *   Runs on the handle's stream. */
nep_status nep_backward_error_noalloc(nep_split h, int m, const double* lambda,
                                      const void* X, double* eta);

/* Derivatives f_i'(z) (FNEvaluateDerivative, Section 3.2.2) for the ell
 * functions at m host points: out[i*m + k] (host, ell*m complex).  Points on
 * a pole or cut give NEP_ERR_NOT_HOLOMORPHIC. */
nep_status nep_fn_eval_derivative(nep_split h, int m, const double* z, double* out);

/* Values f_i(z) for ell functions at m host points (complex): out[i*m + k]
 * (host, ell*m complex).  Points on a pole or cut give NEP_ERR_NOT_HOLOMORPHIC. */
nep_status nep_fn_eval(nep_split h, int m, const double* z, double* out);

/* ------------------------------------------------------------------------ */
/* NLEIGS: rational interpolation and Krylov (Section 4.5)                   */
/* ------------------------------------------------------------------------ */

/* The interpolant R_d(z) = sum_j b_j(z) D_j of eq. (nleigsq) in the rational
 * Newton basis of eq. (nleigsbj) (b_0 = 1, each b_j scaled to maximum modulus
 * 1 on the discretized boundary), with D_j = sum_i d_i^j A_i (eq.
 * (nleigsdsplit)).  Nodes and poles are Leja--Bagby points (eq.
 * (nleigsleja)): sigma_0 is the boundary point at angle 0 of the region g
 * (the target set), the boundary is discretized at npts points
 * c + rho (cos t + i v sin t), t = 2 pi k / npts, and the poles are chosen
 * among the nxi given points of the singularity set (each at most once; the
 * rest infinite).  Greedy ties go to the lowest index within a relative 1e-10.
 * The scalar divided differences d_i^j follow the interpolation conditions of
 * eq. (nleigsdd); the degree d is the first j >= 2 with
 * max_i |d_i^j| < tol max_i |d_i^0| (at most dmax), and the last pole is then
 * set to infinity (the form of eq. (nleigsmatlin)). */
typedef struct {
  double sigma[2];  /* shift of the shift-and-invert Arnoldi (eq. (nleigssinvert)) */
  int k;            /* Arnoldi steps, 1..256                                  */
  int dmax;         /* largest degree, 2..100 (0: 50)                         */
  int npts;         /* boundary points, 8..16384 (0: 1024)                    */
  double tol;       /* degree tolerance (0: 1e-12)                            */
  int nxi;          /* points of the singularity set (0: every pole infinite) */
  const double* xi; /* host, nxi complex                                       */
  double eta_tol;   /* pairs returned have backward error <= eta_tol (0: 1e-10) */
  int max_eigs;     /* capacity of lambda, X and eta (>= 1)                   */
} nep_nleigs_opts;

typedef struct {
  int d;            /* interpolation degree                                   */
  int met;          /* 1 if the degree test was met (else d = dmax)           */
  int k_done;       /* Arnoldi steps taken (fewer than k on an invariant subspace) */
  int basis;        /* columns of the TOAR basis U (k_done + d unless a new
                       vector was linearly dependent)                          */
  double h_last;    /* |h_{k+1,k}|                                            */
  float ms_lu;      /* device time of the assembly and LU of R_d(sigma)       */
  float ms_krylov;  /* wall time of the Arnoldi steps                         */
  float ms_total;   /* wall time of the call                                  */
} nep_nleigs_info;

/* The interpolant alone: d, met, and host arrays of dmax+1 entries (entries
 * beyond d are zero): sigma (complex), xi (complex; an infinite pole has an
 * infinite real part, xi[0] is unused), beta (real), and dd (ell x (dmax+1)
 * complex, d_i^j at dd[i*(dmax+1) + j]).  Evaluates the f_i at the nodes on
 * the device (synchronous).  NEP_ERR_NOT_HOLOMORPHIC if a node lies on a
 * pole or cut of some f_i. */
nep_status nep_nleigs_interp(nep_split h, const nep_contour* g, const nep_nleigs_opts* o, int* d, int* met,
                             double* sigma, double* xi, double* beta, double* dd);

/* Eigenpairs of T inside the region g near the shift, by NLEIGS: the
 * interpolant above, one complex FP64 factorization of R_d(sigma) on the
 * device, and k steps of Arnoldi on (A - sigma B)^{-1} B of the
 * linearization pencil (A, B) of eq. (nleigsmatlin) in the TOAR
 * representation (Algorithm "Arnoldi for NLEIGS with TOAR representation",
 * eqs. (nleigs-toar1)--(nleigs-toar4); classical Gram--Schmidt with one
 * reorthogonalization).  No restart.  Ritz values lambda = sigma + 1/theta of
 * the k x k Hessenberg matrix inside g whose Ritz vectors x (the first block,
 * 2-norm 1, largest entry real positive) have backward error (eq.
 * (sressplit), infinity norms) <= eta_tol are returned, sorted by real then
 * imaginary part.
 *   W0: device, complex n x dmax column-major: the first d columns are the d
 *       parts w^0..w^{d-1} of the starting vector (they must be linearly
 *       independent).
 *   m: number returned (<= max_eigs); lambda: host, 2*max_eigs doubles;
 *   X: device, complex n x max_eigs column-major; eta: host, max_eigs.
 *   H: optional host (k+1) x k complex column-major: the Hessenberg matrix
 *      (columns beyond k_done are zero).  info: optional.
 * Synchronous, on the handle's stream.  Allocates device memory (the factors
 * of one matrix, the basis: n x (d + k + 1) complex). */
nep_status nep_nleigs(nep_split h, const nep_contour* g, const nep_nleigs_opts* o, const void* W0, int* m,
                      double* lambda, void* X, double* eta, double* H, nep_nleigs_info* info);

/* nep_nleigs over nprob problems at once: every problem's own interpolant,
 * shift and starting block, with the factorizations of the R_d(sigma_p) in
 * one batched complex FP64 LU and each Arnoldi step's solves for all problems
 * in one batched solve (the moment plan's kernels over one node per problem);
 * the split products, Gram--Schmidt and Ritz vectors are batched over the
 * problems too.  The pairs returned per problem are those nep_nleigs returns.
 *   h, g, o, W0, X: arrays of nprob (1..4096); o[p].k and o[p].max_eigs must
 *     equal o[0]'s.  W0[p]: device, complex n_p x dmax_p (as in nep_nleigs).
 *   m: host, nprob ints.  lambda: host, 2 * nprob * max_eigs doubles, problem
 *     p's at lambda + 2 p max_eigs.  eta: host, nprob * max_eigs, problem p's
 *     at eta + p max_eigs.  X[p]: device, complex n_p x max_eigs.
 *   info: optional, nprob entries (the ms fields are the whole call's).
 * Errors name the problem.  Runs on the first handle's stream; synchronous.
 * Allocates device memory. */
nep_status nep_nleigs_batch(int nprob, const nep_split* h, const nep_contour* g, const nep_nleigs_opts* o,
                            const void* const* W0, int* m, double* lambda, void* const* X, double* eta,
                            nep_nleigs_info* info);

/* ------------------------------------------------------------------------ */
/* Batched moments: many problems of uneven n in one plan                    */
/* ------------------------------------------------------------------------ */

typedef struct nep_batch_s* nep_batch;

/* Plans the moments of nprob problems sharing (N, L, K, prec) into one set of
 * batched launches over every (problem, node) pair, sorted by size, and
 * captures the launch sequence in a HIP graph.  V[p] and S[p] are device
 * buffers as in nep_ciss_moments; they are bound to the plan (the graph reads
 * and writes exactly these buffers on every run).
 *   use_graph: 1 = capture and replay a HIP graph, 0 = eager launches. */
nep_status nep_batch_create(int nprob, const nep_split* h,
                            const nep_contour* g, const nep_ciss_opts* o,
                            const void* const* V, void* const* S,
                            int use_graph, void* stream, nep_batch* out);

/* Runs the plan.  st (optional, nprob entries) as in nep_ciss_moments; if
 * non-NULL the call is synchronous (it ends with nep_batch_wait).  If NULL it
 * returns after enqueueing; nep_batch_wait must then follow before the
 * moments are used: the run does a fixed number of refinement sweeps on the
 * device, and nodes still above the tolerance are re-solved in FP64 there. */
nep_status nep_batch_run(nep_batch b, nep_ciss_stats* st);

/* Waits for the last nep_batch_run, re-solves in FP64 the nodes its sweeps
 * left above the refinement tolerance (mixed precision with fp64_fallback),
 * and reports per-problem stats in st (optional, nprob entries) and the
 * status: the most severe of NEP_ERR_NOT_HOLOMORPHIC, NEP_ERR_SINGULAR,
 * NEP_ERR_REFINE over the problems.  NEP_ERR_ARG if no run is pending. */
nep_status nep_batch_wait(nep_batch b, nep_ciss_stats* st);

nep_status nep_batch_destroy(nep_batch* b);

/* One-shot: create, run synchronously, destroy. */
nep_status nep_ciss_moments_batch(int nprob, const nep_split* h,
                                  const nep_contour* g, const nep_ciss_opts* o,
                                  const void* const* V, void* const* S,
                                  nep_ciss_stats* st);

/* ------------------------------------------------------------------------ */
/* Serving: "eigenvalues inside this contour" queries, continuous batching   */
/* ------------------------------------------------------------------------ */

typedef struct nep_server_s* nep_server;

typedef struct {
  long long hbm_budget;  /* bytes of device memory the server may hold for
                            per-query workspaces (factors, solves, moments)   */
  int max_inflight;      /* queries on the device at once (>= 1)              */
  int nstreams;          /* device streams used to overlap queries (>= 1)     */
} nep_server_opts;

typedef struct {
  int status;            /* nep_status of the query                            */
  int m;                 /* eigenpairs returned                                */
  int n_inside;          /* of which inside the contour                        */
  int reused;            /* 1: ran on resident factors (no assembly or LU)     */
  double t_submit, t_start, t_done;  /* seconds on the server clock            */
  int L_used;            /* probe columns in the final moments (L, or more     */
                         /* after augmentation from a probe pool)              */
} nep_query_info;

nep_status nep_server_create(const nep_server_opts* o, nep_server* out);

/* Factors stay resident after a query completes, keyed by (handle,
 * contour, N, L, K, precision, refinement options).  A later query with the
 * same key runs on them: its probes are solved, refined and reduced to
 * moments without assembling or factoring T again (the results are those a
 * new factorization would give, bit for bit), and its info reports
 * reused = 1.  Queued queries with the key of one already dispatched wait for
 * its factors instead of factoring the same matrices again.  Resident
 * factors count against hbm_budget and are evicted least recently used when
 * a new batch needs the room; those of a destroyed handle are never used
 * again (handles carry a process-unique id) and are freed on eviction or by
 * nep_server_destroy.  A handle must stay alive while it has queries queued
 * or running. */

/* Queues a query: moments and extraction of h inside g.
 *   V: host, complex n x L column-major (copied before the call returns).
 *   Results are written to the host arrays lambda (2*max_eigs), eta
 *   (max_eigs), inside (max_eigs) and, if X is non-NULL, to host X
 *   (complex n x max_eigs), when the query completes; they must stay valid
 *   until then.  *ticket identifies the query.
 * Returns NEP_ERR_BUSY only if the query can never fit the HBM budget. */
nep_status nep_server_submit(nep_server s, nep_split h, const nep_contour* g,
                             const nep_ciss_opts* o, const nep_extract_opts* e,
                             const void* V, double* lambda, double* eta,
                             int* inside, void* X, long long* ticket);

/* As nep_server_submit, with a probe pool for rank saturation (Section 2:
 * the moments resolve at most K*L eigenvalues; the count of eigenvalues
 * inside is the number of roots of det T(z) there, eq. (nep)).
 *   V: host, complex n x Lmax column-major, Lmax a multiple of L, at most
 *   256 and at most n (copied before the call returns).  The query runs on
 *   the first L columns; while its extraction finds the moment rank equal
 *   to K*L_used and columns are left, the next L columns are solved on the
 *   same factors (no assembly or LU), their moments join the others and the
 *   extraction runs again on all L_used columns, as nep_eigs does on a
 *   handle.  nep_query_info.L_used reports the columns used.  The rank can
 *   reach K*L_used, so max_eigs of K*Lmax holds every case (a larger rank
 *   than max_eigs ends the query with NEP_ERR_ARG).  Lmax = L is
 *   nep_server_submit. */
nep_status nep_server_submit_pool(nep_server s, nep_split h, const nep_contour* g,
                                  const nep_ciss_opts* o, const nep_extract_opts* e,
                                  const void* V, int Lmax, double* lambda, double* eta,
                                  int* inside, void* X, long long* ticket);

/* Non-blocking: returns 1 in *done when the query has finished. */
nep_status nep_server_poll(nep_server s, long long ticket, int* done,
                           nep_query_info* info);

/* Blocks until the query has finished. */
nep_status nep_server_wait(nep_server s, long long ticket, nep_query_info* info);

/* Current clock of the server (seconds), for latency accounting. */
double nep_server_clock(nep_server s);

/* Drains every queued query and frees the server. */
nep_status nep_server_destroy(nep_server* s);

/* ------------------------------------------------------------------------ */

/* ------------------------------------------------------------------------ */
/* Autotuning of launch shapes                                              */
/* ------------------------------------------------------------------------ */

/* Not an operation of the paper: batching every (problem, node) pair of the
 * moment stage into shared launches leaves a few launch-shape choices whose
 * best setting depends on the batch and the device.  Every setting computes
 * the moments to the same accuracy; all but the panel width also give the same
 * bits (the panel width changes the rounding of the factors).  One setting: */
typedef struct {
  int lg;        /* right-hand columns per work-group of the triangular solves (4, 8 or 16) */
  int paired;    /* large matrices as paired 256-thread solve groups: -1 when they make at
                    least 2048 groups, 0 never, 1 always (complex FP32, lg <= 8, n <= 1024) */
  int small_min; /* panels of at most 256 rows take 256-thread groups (two per CU) when at
                    least small_min of them share an LU step (0 always; INT_MAX never) */
  int early_fork; /* the rest of an LU step's update starts on a second stream as soon as the
                     panel is done (1) or after the next panel's columns are updated (0);
                     -1: built in (1 for 64-wide complex-FP32 panels, else 0) */
  int jb;        /* LU panel width, 64 or 128 (built in: 128 when every matrix of the plan
                    has at least 2048 rows) */
  float ms;      /* median device time of one full moment pass with this setting */
} nep_tune_cand;

/* on = 1: every moments plan built afterwards (the plan of a nep_ciss_moments
 * call whose shapes differ from the handle's last call, and nep_batch_create's,
 * before its graph is captured) first times each candidate setting with reps
 * full moment passes on its own buffers and the call's stream (so S is written
 * more than once; the call then runs as usual) and keeps the fastest.  on = 0
 * (the default): the built-in choice.  Either way a setting chosen earlier in
 * the process for a plan with the same launch shapes (precision, N, L,
 * sweeps, the multiset of sizes) is applied without timing.  Process-wide.
 * Timing synchronizes the call's stream, so a call that builds a plan with
 * tuning on must not be made while that stream is being captured into a graph
 * (the HIP error is returned as NEP_ERR_DEVICE).
 * Errors: NEP_ERR_ARG if reps is outside 1..64. */
nep_status nep_tune_set(int on, int reps);

/* The last plan built: *ncand candidates timed (0 when the setting came from
 * the cache, with *cached = 1, or when tuning was off, with *cached = 0 and
 * *chosen = -1), the index of the one kept in *chosen, and the first
 * min(max, *ncand) of them in cand (host array).  A plan with a single
 * candidate reports it with ms = 0.  Errors: NEP_ERR_ARG on null outputs. */
nep_status nep_tune_report(int max, nep_tune_cand* cand, int* ncand, int* chosen, int* cached);

/* Forgets every cached setting. */
nep_status nep_tune_clear(void);

/* ------------------------------------------------------------------------ */
/* Instrumentation                                                           */
/* ------------------------------------------------------------------------ */

/* Enables (1) or disables (0) HIP-event timing of every trailing-update GEMM
 * launch of the LU (k_lu_gemm_c64 / k_lu_gemm_c128) on the stream it runs on,
 * and around nep_nleigs's solve and split-product launches.
 * Enabling clears earlier records.  Process-wide; not thread-safe. */
nep_status nep_prof_enable(int on);

/* Reads the records: for kind 0 (complex FP32 GEMM) or 1 (complex FP64 GEMM),
 * *launches = number of launches, *ms = summed device time of the launches
 * (synchronizes their events), *flops = summed algorithmic flops of the
 * launches (8 real flops per complex multiply-add).  Kinds 2 and 3 record
 * nep_nleigs's triangular-solve launches (one per triangle) and split-form
 * product launches; for them *flops holds the summed algorithmic HBM bytes
 * (the factor triangle outside its diagonal blocks, the diagonal-block
 * inverses and the vectors; every A_i once and the vectors). */
nep_status nep_prof_read(int kind, int* launches, double* ms, double* flops);

/* Thread-local description of the last error on the calling thread. */
const char* nep_last_error(void);

/* Library version string. */
const char* nep_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NEP_H */
