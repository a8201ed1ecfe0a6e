/*
 * kcpc.h - C ABI of an MI355X (gfx950) solver for the kernel-compensated Yee-scheme
 * Maxwell eigenproblem of 3D photonic crystals with anisotropic permittivity
 * (Jin & Xie, "A Robust GPU-Accelerated Kernel Compensation Solver with Novel
 * Discretization for Photonic Crystals in Anisotropic Media").
 *
 * Problem.  For a simple-cubic unit cell with grid division N (h = 1/N), a piecewise
 * constant Hermitian inverse permittivity and a Bloch wave vector k, find the m smallest
 * strictly positive eigenvalues lambda = omega^2 of
 *
 *     Op = A M A^H + gamma B^H B                                   (Section 2.3, eq (2.13))
 *
 * with A the Yee curl and B the divergence of eqs (2.5)-(2.7), M the discrete inverse
 * permittivity (eq (3.3) diagonal, eq (3.4) "Trivial", eq (3.8) "CrossDoF") and gamma the
 * penalty of eq (2.26).  The library works on k-space coefficients x = F3^H H (eq (2.30)),
 * where F3 applies the unitary DFT of Lemma 2.1 (omega = exp(+2 pi i/N)) to each of the
 * three face components; in those coordinates Op becomes
 *
 *     K_A F3^H M F3 K_A^H + gamma K_B                               (Prop 2.8, eq (2.30))
 *
 * with K_A, K_B diagonal per frequency.
 *
 * Vector layout.  A block of nvec vectors is complex128 (interleaved re, im), laid out
 * [nvec][3][N][N][N] with the k-space index (qz, qy, qx), qx fastest; frequency index q
 * corresponds to theta_q = 2 pi q / N.  Unless a function says otherwise vector pointers
 * are DEVICE pointers owned by the caller; "_host" arguments are host pointers.
 *
 * Streams.  Every call that touches the GPU takes a hipStream_t passed as void* (NULL is
 * the default stream) and enqueues its work there; calls return after enqueueing, except
 * kc_solve which returns when the solve is complete.
 *
 * Errors.  Every function returns a kc_status; on error kc_last_error() gives a message
 * (per calling thread).  No C++ exception crosses this boundary.  A handle is not
 * thread-safe.
 *
 * Memory.  The library owns the handle and its device workspaces (allocated on first use,
 * grown as needed, released by kc_destroy).  Workspace memory comes from the allocator
 * callbacks given to kc_create (e.g. a framework's caching allocator), or from hipMalloc /
 * hipFree when none are given.
 */
#ifndef KCPC_H
#define KCPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum kc_status {
  KC_OK = 0,
  KC_ERR_INVALID_ARG = 1,   /* bad pointer, size or index                               */
  KC_ERR_UNSUPPORTED = 2,   /* N is not a supported FFT length (see kc_supported_n)    */
  KC_ERR_NOT_HPD = 3,       /* inverse-permittivity table violates Assumption 3.1      */
  KC_ERR_HIP = 4,           /* a HIP runtime call or kernel launch failed              */
  KC_ERR_ALLOC = 5,         /* device allocation failed                                */
  KC_ERR_NO_CONVERGENCE = 6,/* kc_solve hit maxit; outputs hold the best iterate       */
  KC_ERR_BREAKDOWN = 7      /* non-finite values or loss of positive definiteness      */
} kc_status;

/* Discretisation of the inverse permittivity (Section 3). */
enum {
  KC_EPS_DIAGONAL = 0, /* eq (3.3): diagonal entries at edge points, off-diagonals ignored   */
  KC_EPS_TRIVIAL = 1,  /* eq (3.4): off-diagonal entries at volume points, no interpolation  */
  KC_EPS_CROSSDOF = 2  /* eq (3.8): symmetrised cross-DoF transfer (four-point averages)     */
};

/* Arithmetic of the operator application (FFTs, curl, permittivity). */
enum { KC_PREC_FP64 = 0, KC_PREC_FP32 = 1 };

typedef struct kc_op kc_op;

/* Caller allocator for the device workspaces of a handle: alloc returns `bytes` of device
 * memory on the current device (NULL on failure), free releases a pointer alloc returned
 * (with the same byte count).  Both are called from the thread that calls the library, never
 * during a hipGraph capture, and free only after the library has synchronised the device. */
typedef void* (*kc_alloc_fn)(void* ctx, size_t bytes);
typedef void (*kc_free_fn)(void* ctx, void* ptr, size_t bytes);

/* Properties of a handle found by kc_create (bits of kc_op_flags). */
enum {
  /* Gershgorin's bound does not prove the discrete inverse permittivity M positive definite:
   * some row's diagonal does not exceed the sum of the moduli of its off-diagonal entries
   * (strict diagonal dominance, the sufficient condition behind Props 3.8 and 3.10; for
   * Trivial, the rows of eq (3.4)).  M may still be HPD; the solver runs anyway. */
  KC_FLAG_HPD_UNPROVEN = 1
};

/* Per-k-point warnings (bits of kc_kpoint_flags). */
enum {
  /* some |k_i| > pi: the lower bound of Lemma 2.4 (2) on the spectrum of the penalty term
   * (eq (2.20)) and with it the guarantee of the gamma rule, eq (2.26), is not given */
  KC_KFLAG_K_OUTSIDE = 1,
  /* after the last kc_solve: lambda_m >= gamma * s_min (kc_spurious_bound), so a computed
   * eigenvalue may belong to the penalty term's spurious spectrum (Prop 2.3, Remark 2.6);
   * a larger gamma (kc_set_kpoints) separates them */
  KC_KFLAG_SPURIOUS_RISK = 2
};

/* 1 if N is a supported grid division (FFT length), else 0.  Supported: 4, 6, 8, 12, 16,
 * 24, 32, 48, 64, 96, 128. */
int kc_supported_n(int N);

/*
 * Create an operator for grid division N and an inverse-permittivity field.
 *   lattice_host : NULL (simple cubic) or float64 [3][3], the primitive lattice vectors a_1,
 *                  a_2, a_3 as rows (lattice constant 1; e.g. FCC, BCC of eq (4.1)).  The grid is
 *                  the unit cube of fractional coordinates (the coordinate transform of
 *                  Section 2.2): the point of index (i, j, k) sits at x = sum_r xi_r a_r, and the
 *                  difference blocks become sum_j b_ji D_{1,j} + i k_i D_{0,i}, b = A^{-1},
 *                  A = (a_1 a_2 a_3) (eq (2.12), the sum taken over the axis of D_1).  Wave
 *                  vectors stay Cartesian.  Dependent vectors: KC_ERR_INVALID_ARG.
 *   stencil_m    : 1..5, order 2m of the finite-difference stencils of the curl and
 *                  divergence (eq (2.34), coefficients from eq (2.35), Table 1); 1 is the
 *                  second-order Yee scheme of eq (2.5).  The cross-DoF transfer T of eq (3.7)
 *                  keeps its two-point average at every order.
 *   eps_scheme   : KC_EPS_DIAGONAL / KC_EPS_TRIVIAL / KC_EPS_CROSSDOF.
 *   mat_ids_host : uint8 [4][N^3] material ids of the x-edge, y-edge, z-edge and volume
 *                  points (eqs (2.1)-(2.3), eq (3.2)); index i + N j + N^2 k.  The points of
 *                  cell (i, j, k) are ((i-1/2)h, jh, kh), (ih, (j-1/2)h, kh),
 *                  (ih, jh, (k-1/2)h) and ((i-1/2)h, (j-1/2)h, (k-1/2)h).
 *   eps_inv_host : float64 [n_mat][3][3][2]: the complex inverse permittivity of each
 *                  material (row-major, (re, im)); must be Hermitian with eigenvalues in
 *                  (0, 1] (Assumption 3.1), else KC_ERR_NOT_HPD.  Material 0 is usually air.
 *   alloc, free_fn, alloc_ctx : caller allocator of every device buffer the handle owns
 *                  (both NULL: hipMalloc / hipFree; exactly one NULL is KC_ERR_INVALID_ARG).
 *   stream       : stream of the uploads (the call returns when they are complete).
 * The ids and the table are copied; the caller keeps ownership of its buffers.  Every argument
 * is checked before any device work.  kc_op_flags reports whether M was proven HPD.
 */
int kc_create(int N, const double* lattice_host, int stencil_m, int eps_scheme, const uint8_t* mat_ids_host,
              int n_mat, const double* eps_inv_host, kc_alloc_fn alloc, kc_free_fn free_fn, void* alloc_ctx,
              void* stream, kc_op** out);

/* KC_FLAG_* bits of a handle (0: M proven HPD by Gershgorin's bound). */
int kc_op_flags(const kc_op* op, int* flags_host);

/*
 * Set the Bloch wave vectors (Cartesian, lattice constant 1): k_host float64 [nk][3].
 * gamma_host: float64 [nk] penalty coefficients, or NULL for the rule of Remark 2.6,
 * eq (2.26) (4 pi^2 if k = 0 or |k| >= 1, else 4 pi^2 / |k|^2).  Every k and gamma is checked
 * (finite; gamma > 0) before the handle changes: a rejected call leaves the previous k-points in
 * place.  A k-point with some |k_i| > pi is accepted with KC_KFLAG_K_OUTSIDE set.
 */
int kc_set_kpoints(kc_op* op, int nk, const double* k_host, const double* gamma_host);

/* Penalty coefficients in use: gamma_host float64 [nk]. */
int kc_get_gamma(const kc_op* op, double* gamma_host);

/* KC_KFLAG_* bits of every k-point: flags_host int32 [nk]. */
int kc_kpoint_flags(const kc_op* op, int* flags_host);

/*
 * gamma_k * s_min(k) per k-point (float64 [nk]): s_min is the smallest positive eigenvalue of
 * the penalty term's symbol, min over frequencies p of |K_1(q_x)|^2 + |K_2(q_y)|^2 + |K_3(q_z)|^2
 * with s(p) > 0 (|k|^2 for k != 0 with the second-order stencils, Lemma 2.4 (2)).  By Prop 2.3
 * the spurious eigenvalues of Op are gamma s(p) >= this bound, so computed eigenvalues below it
 * are physical.
 */
int kc_spurious_bound(const kc_op* op, double* bound_host);

/*
 * y = Op_k x for nvec vectors (k-space coefficients, eq (2.30)).  Vector v uses the k-point
 * ik0 + v / vecs_per_k (vecs_per_k >= 1; use vecs_per_k = nvec for a single k-point).
 *   x, y : device complex128 [nvec][3][N^3]; x and y must not overlap.
 *   prec : KC_PREC_FP64, or KC_PREC_FP32 (FFTs, curl and permittivity in FP32; the penalty
 *          term and the result are accumulated in FP64).
 */
int kc_apply(kc_op* op, int ik0, int nvec, int vecs_per_k, const void* x, void* y, int prec,
             void* stream);

/*
 * kc_apply with HIP events recorded on `stream` between its pencil passes (for measuring
 * each pass): pass_ms_host float64 [6] receives the milliseconds of the passes in launch order
 * (CrossDoF: X1, Y1, Za, Zb, Y2, X2; otherwise X1, Y1, Z, Y2, X2), *npass_host their count.
 * Blocks until the application is complete.  Same arguments and errors as kc_apply.
 */
int kc_apply_timed(kc_op* op, int ik0, int nvec, int vecs_per_k, const void* x, void* y, int prec,
                   void* stream, double* pass_ms_host, int* npass_host);

/*
 * z = K_P^{-1} r, the diagonal-block preconditioner of eqs (2.31)-(2.32), per frequency:
 * K_P = K_A K_A^H + gamma K_B.  Where K_P is singular (the DC frequency at k = 0, whose
 * modes are the constant fields of Prop 2.5) z is zero.  r, z: device complex128
 * [nvec][3][N^3]; r == z is allowed.
 */
int kc_precond(kc_op* op, int ik0, int nvec, int vecs_per_k, const void* r, void* z,
               void* stream);

/*
 * Block kernels of the LOBPCG iteration (Section 4, the custom block solver; run by kc_solve,
 * exposed for testing and measurement).  A block holds, for each of nb k-points b, nc columns
 * of n complex128 entries, column j of k-point b at offset (b * nc + j) * n (entries).
 *
 * kc_block_work_bytes: device workspace (bytes) that kc_block_gram and kc_block_update need
 * for nb k-points, n rows and at most nc columns (0 for arguments out of range).
 */
size_t kc_block_work_bytes(int nb, size_t n, int nc);

/*
 * Gram matrices of the search space: GA_b = S_b^H AS_b and GB_b = S_b^H S_b, each nc x nc,
 * row-major, G_b[i][j] = sum_r conj(S_b[r][i]) AS_b[r][j] (resp. S_b[r][j]).  Both are taken
 * to be Hermitian: AS_b must be the image A S_b of S_b under a Hermitian A (as in LOBPCG);
 * the 16 x 16 tiles on and above the diagonal are summed, the others are their conjugates.
 *   S, AS : device complex128, nb blocks of nc columns (1 <= nc <= 96; above 64 the kernels
 *           stage 80 or 96 columns, as for the solver's blocks of more than 21 columns)
 *   GA, GB: device complex128 [nb][nc][nc]
 *   work  : device scratch of at least kc_block_work_bytes(nb, n, nc) bytes
 * The partial sums over row chunks are added in a fixed order (results are reproducible).
 */
int kc_block_gram(int nb, size_t n, int nc, const void* S, const void* AS, void* GA, void* GB, void* work,
                  size_t work_bytes, void* stream);

/*
 * kc_block_gram for callers that cannot allocate device memory (code under hipGraph capture,
 * tight serving loops, harnesses that forbid allocation): no workspace argument and no
 * allocation; the partial sums live in a fixed static device array of KC_NOALLOC_SCRATCH_BYTES
 * (32 MiB) per GPU, held until the process ends.  Same arguments, layout and results as
 * kc_block_gram (up to the order of the partial sums: fewer, longer row chunks when the array
 * would not hold the usual number).  Sizes with nb * ceil(nc/16) * (ceil(nc/16) + 1) * 4096 >
 * KC_NOALLOC_SCRATCH_BYTES (e.g. nb > 409 at nc > 48) give KC_ERR_INVALID_ARG before any device
 * work.  Every call on a GPU uses that GPU's one array, so calls that overlap on one GPU (other
 * streams, other threads) race; the array needs no clearing (each call writes every partial sum
 * before it reads it).
 */
#define KC_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
int kc_block_gram_noalloc(int nb, size_t n, int nc, const void* S, const void* AS, void* GA, void* GB,
                          void* stream);

/*
 * One Rayleigh-Ritz update with the next residuals (eq (4.3)), in place.  Per k-point b the
 * block holds 3mb columns S_b = [X W P] and AS_b = [AX AW AP] (1 <= mb <= 32), and
 * C_b = [C1 | Cp] is 3mb x 2mb (row-major, complex128 [nb][3mb][2mb]):
 *   X <- S_b C1, P <- S_b Cp, AX <- AS_b C1, AP <- AS_b Cp   (W and AW are left as they are)
 *   R_j = AX_j - theta_j X_j          (new X, AX; R device complex128 [nb * mb][n])
 *   res_j = |R_j| / |X_j| (0 where X_j = 0), xnorm2_j = |X_j|^2    (device double [nb * mb])
 * theta: device double [nb * mb].  S, AS and R must not overlap.  work as for kc_block_gram.
 */
int kc_block_update(int nb, size_t n, int mb, void* S, void* AS, const void* C, const double* theta, void* R,
                    double* res, double* xnorm2, void* work, size_t work_bytes, void* stream);

/*
 * Real-space face fields of k-space coefficients, H = F3 x (eq (2.30), Lemma 2.1): per component
 * H[j] = N^{-3/2} sum_q x[q] exp(+2 pi i (j . q) / N).  x, H: device complex128 [nvec][3][N^3]
 * (H in the index order i + N j + N^2 k of the face points of eqs (2.1)-(2.3)); x == H is
 * allowed.  kc_to_kspace is the inverse, x = F3^H H.
 */
int kc_to_real_space(kc_op* op, int nvec, const void* x, void* H, void* stream);
int kc_to_kspace(kc_op* op, int nvec, const void* H, void* x, void* stream);

/*
 * Unnormalised 3D DFT of nvec scalar grids along x, y and z:
 *   out[q] = sum_j in[j] exp(sign 2 pi i (j . q) / N), sign = +1 or -1.
 * prec KC_PREC_FP64: in/out complex128 [nvec][N^3]; KC_PREC_FP32: complex64.  in == out is
 * allowed.  (The building block of kc_apply, exposed for testing.)
 */
int kc_fft3d(int N, int nvec, int sign, int prec, const void* in, void* out, void* stream);

/*
 * z = T_E r, the transverse-projection preconditioner (not part of the paper's method; the
 * classical planewave choice of Johnson & Joannopoulos, Opt. Express 8 (2001) 173, carried over
 * to the operator of Prop 2.8):
 *   T_E = K_A^{+H} F3^H E F3 K_A^{+} + (gamma K_B)^{+}
 * with K_A, K_B of eq (2.29), ^+ the Moore-Penrose pseudo-inverse per frequency, and E a
 * positive diagonal field on the edge points (component c scales the c-edge values).  Since
 * K_A^{+} = K_A^H / s with s = |K_1|^2 + |K_2|^2 + |K_3|^2, it costs one pass over the
 * operator's FFT pipeline.  With E = 1 it equals K_P^{-1} (kc_precond); with E = eps^{-1}
 * pointwise inverted it inverts Op exactly for a homogeneous isotropic medium.
 *   efield : NULL for E_c = 1/(eps^-1)_cc at the c-edge points, or device float32
 *            [nk_used][3][N^3] with one field per k-point of the call (nk_used =
 *            (nvec - 1) / vecs_per_k + 1)
 *   prec   : KC_PREC_FP64 or KC_PREC_FP32 arithmetic of the transforms
 * r, z: device complex128 [nvec][3][N^3], must not overlap.  Zero where K_P is singular.
 */
int kc_precond_transverse(kc_op* op, int ik0, int nvec, int vecs_per_k, const void* r, void* z,
                          const float* efield, int prec, void* stream);

/*
 * Gradient of sum_j w_j Re<e_j, T_E r_j> with respect to the field E, accumulated (+=) into
 * g (device float32 [nvec / vecs_per_k][3][N^3], one field per k-point): for training the
 * learned field.  r, e device complex128 [nvec][3][N^3]; w device float64 [nvec].
 */
int kc_tp_grad(kc_op* op, int ik0, int nvec, int vecs_per_k, const void* r, const void* e,
               const double* w, float* g, void* stream);

/* Preconditioner of kc_solve: the diagonal-block K_P^{-1} of eqs (2.31)-(2.32), T_E with the
 * learned field (needs kc_attach_net; a k-point whose residuals stall falls back to K_P^{-1}),
 * or T_E with E_c = 1/(eps^-1)_cc. */
enum { KC_PRECOND_DIAG = 0, KC_PRECOND_LEARNED = 1, KC_PRECOND_TRANSVERSE = 2 };

/* Solver options for kc_solve (LOBPCG with soft locking, Section 4). */
typedef struct kc_solve_opts {
  int m;              /* bands wanted (smallest positive eigenvalues)                      */
  int guard;          /* extra block columns carried but not required to converge (>= 0); */
                      /* m + guard <= 32 (blocks of more than 21 columns take the wide    */
                      /* kernels: Rayleigh-Ritz matrices in global memory)                 */
  double tol;         /* convergence: Res_j = ||Op x_j - lambda_j x_j|| / ||x_j|| <= tol  */
                      /* (eq (4.3)), checked with an FP64 operator application             */
  int maxit;          /* iteration limit                                                   */
  int prec;           /* KC_PREC_FP64, or KC_PREC_FP32: FP32 operator applications until   */
                      /* the residuals reach switch_tol, stall (no 30 % progress in 4      */
                      /* iterations) or first rise within 10x the FP32 rounding floor     */
                      /* 2^-24 s_max |eps^-1|; FP64 from there on                          */
  double switch_tol;  /* residual level where FP32 applications stop (prec = FP32)         */
  int batch_k;        /* k-points solved together in one set of launches (>= 1)            */
  uint64_t seed;      /* seed of the random initial block                                  */
  int verbose;        /* 1: print per-iteration residuals to stderr                        */
  int precond;        /* KC_PRECOND_DIAG, _TRANSVERSE or _LEARNED (needs kc_attach_net)    */
  int graph;          /* 1: capture each iteration's launches (preconditioner, operator,   */
                      /* Rayleigh-Ritz, update, residuals) once per precision in a hipGraph */
                      /* and replay it, on a private stream; 0: launch them one by one      */
  const void* x_init; /* NULL: seeded random start.  Else device complex128 [nk][m][3N^3]:   */
                      /* start vectors per k-point (e.g. the converged fields of the        */
                      /* neighbouring k-points of a path, kc_solve's X_out); they enter the */
                      /* first search directions next to the random guard columns.  At k = 0 */
                      /* their constant (DC) part is removed (Prop 2.5 (1)).  Not modified. */
  int start;          /* without x_init: KC_START_RANDOM (K_P^{-1} applied to a seeded random */
                      /* block) or KC_START_PLANE_WAVES (up to m of the first directions are */
                      /* the lowest transverse plane waves of the k-point: the frequencies q */
                      /* with the smallest |K(q)|^2, s = 0 excluded, two polarizations      */
                      /* orthogonal to conj(K(q)) each, whole groups of equal |K(q)|^2 only;  */
                      /* the modes of a homogeneous medium, eq (2.30) with Lemma 2.4; the   */
                      /* other columns as KC_START_RANDOM)                                   */
} kc_solve_opts;

enum { KC_START_RANDOM = 0, KC_START_PLANE_WAVES = 1 };

/* Fill opts with defaults (m = 10, guard = 0, tol = 1e-8, maxit = 500, FP64, batch_k = 1,
 * diagonal-block preconditioner, graph = 1, random start). */
void kc_solve_opts_default(kc_solve_opts* opts);

/*
 * Smallest positive eigenvalues of Op_k for k-points ik0 .. ik0+nk-1.
 *   eig_host   : float64 [nk][m] eigenvalues lambda = omega^2, ascending
 *   res_host   : float64 [nk][m] final residuals Res_j (eq (4.3)), FP64 application
 *   iters_host : int32 [nk] iterations used (may be NULL)
 *   X_out      : NULL, or device complex128 [nk][m][3][N^3] for the eigenvectors
 * At k = 0 the three constant fields (Prop 2.5 (1)) are deflated and not reported.
 * Returns KC_ERR_NO_CONVERGENCE if some k-point did not reach tol within maxit, or stagnated
 * (in the FP64 phase its largest band residual did not halve in 200 iterations, or, once within
 * 1e3 tol, rose above 10 times its best in two successive iterations: what a tol below the
 * rounding floor of the operator's FP64 application leads to); the outputs then hold that
 * k-point's last iterate.
 */
int kc_solve(kc_op* op, int ik0, int nk, const kc_solve_opts* opts, double* eig_host,
             double* res_host, int* iters_host, void* X_out, void* stream);

/* Statistics of the last kc_solve: float64 [8] = {matvecs FP64 (vector count), matvecs FP32,
 * seconds total, iterations (sum over k-points), k-points that kept the transverse or learned
 * preconditioner to the end, preconditioner applications (vector count), iterations whose Gram
 * step formed only the new directions' columns (the X/P blocks taken from the previous
 * Rayleigh-Ritz step), 0}. */
int kc_last_solve_stats(const kc_op* op, double* stats_host);

/*
 * Residual history of k-point ik0 + k of the last kc_solve (0 <= k < its nk): the largest
 * Res_j (j < m, eq (4.3)) before each iteration, and the precision (KC_PREC_*) of that
 * iteration's operator applications.  res_host float64 [cap], prec_host int32 [cap] (either may
 * be NULL); *count receives the number of iterations recorded (the first min(cap, count) are
 * written).
 */
int kc_last_residual_history(const kc_op* op, int k, double* res_host, int* prec_host, int cap, int* count);

/*
 * Tile widths (pencils per workgroup) chosen for the handle's passes in precision prec, int32
 * [10] in the order X1, Y (inverse), Za, Zb, Z (Trivial/diagonal), Y (forward), X2, then the
 * transverse preconditioner's X1, Z and X2; 0 while not yet chosen.  On a handle's first
 * application in a precision (N >= 32) every valid width of every pass is timed on a block of
 * up to 32 vectors and the fastest kept; smaller grids use a fixed rule.
 */
int kc_tile_widths(const kc_op* op, int prec, int* widths_host);

/* Release the handle's work buffers (the LOBPCG blocks of kc_solve and the operator's
 * intermediates; they are allocated again on the next call that needs them), keeping the
 * geometry, tables and k-points.  Waits for the device first. */
int kc_release_workspaces(kc_op* op);

/* Release the handle and every device buffer it owns.  NULL is allowed. */
void kc_destroy(kc_op* op);

/*
 * Learned preconditioner.  A three-layer periodic 3D convolution network (3x3x3 kernels,
 * 15 -> 32 -> 32 -> 3 channels, leaky ReLU slope 0.01, BF16 weights and activations with FP32
 * accumulation) maps the dielectric structure and the wave vector to the field of T_E
 * (kc_precond_transverse): E_c = E0_c exp(clamp(y_c, -3, 3)) with E0_c = 1/(eps^-1)_cc at the
 * c-edge points and y the network output.  Input channels per cell: the inverse permittivity
 * (9: diagonal at the x/y/z-edge points, Re/Im of the upper off-diagonals at the volume point),
 * log E0 (3) and k/pi (3).  The network runs once per k-point and solve.  Grids need
 * N % 16 == 0.
 *
 * Tensors: network input bf16 [batch][N^3][32] (channels-last, channels 15..31 zero), output
 * float32 [batch][N^3][16] (channels 3..15 zero); parameters float32 in the order
 * W1 b1 W2 b2 W3 b3 with W[co][ci][dz][dy][dx] (tap offsets d-1, circular) and b[co].
 */
typedef struct kc_net kc_net;
int kc_net_create(uint64_t seed, kc_net** out);         /* He-normal init, last layer ~0    */
size_t kc_net_param_count(void);
int kc_net_get_params(const kc_net* net, float* host, size_t n);
int kc_net_set_params(kc_net* net, const float* host, size_t n);
int kc_net_forward(kc_net* net, int N, int batch, const void* in_bf16, void* out_f32, void* stream);
/* Mean-squared-error loss over the 3 output channels and its gradient for every parameter
 * (grads_host float32 [kc_net_param_count()] or NULL to keep them on the device for
 * kc_net_adam_step).  Blocks until done. */
int kc_net_gradients(kc_net* net, int N, int batch, const void* in_bf16, const void* target_f32,
                     double* loss_host, float* grads_host, void* stream);
/* Parameter gradients for a given gradient of a loss with respect to the network output
 * (gout_f32 float32 [batch][N^3][16], channels 3..15 ignored by the weights' padding);
 * grads_host as in kc_net_gradients.  Blocks until done. */
int kc_net_backward(kc_net* net, int N, int batch, const void* in_bf16, const void* gout_f32,
                    float* grads_host, void* stream);
/* One Adam step (Kingma & Ba) with the gradients of the last kc_net_gradients/backward call. */
int kc_net_adam_step(kc_net* net, float lr, float beta1, float beta2, float eps, void* stream);
void kc_net_destroy(kc_net* net);
/* Attach (or detach with NULL) a network to an operator; the operator does not own it. */
int kc_attach_net(kc_op* op, kc_net* net);
/* Network input for k-points ik0 .. ik0+nk-1: feat_bf16 [nk][N^3][32] (no network needed). */
int kc_net_features(kc_op* op, int ik0, int nk, void* feat_bf16, void* stream);
/* Learned field E of k-points ik0 .. ik0+nk-1 with the attached network: float32
 * [nk][3][N^3]. */
int kc_net_efield(kc_op* op, int ik0, int nk, float* efield, void* stream);
/* z = T_E r with the attached network's field (kc_net_efield then kc_precond_transverse). */
int kc_precond_learned(kc_op* op, int ik0, int nvec, int vecs_per_k, const void* r, void* z, int prec,
                       void* stream);

/*
 * Training support of the learned preconditioner (not part of the paper, whose solver uses the
 * diagonal-block K_P^{-1} of eqs (2.31)-(2.32); the network predicts the field E of T_E).  All
 * vectors are device complex128 k-space vectors [nvec][3][N^3] of one k-point ik; the calls run
 * on `stream`, synchronise it before returning, and take their work vectors from the handle's
 * allocator (released by kc_release_workspaces).
 *
 * kc_pcg: c_j = Op^{-1} r_j by conjugate gradients preconditioned with T_E of the classical field
 *   E_c = 1/(eps^-1)_cc, FP64 operator applications, until every recurrence residual satisfies
 *   |r_j - Op c_j| <= tol |r_j|.  r and c must not overlap; c is overwritten.  *iters (host, may
 *   be NULL) receives the iterations done; a zero r_j gives c_j = 0.  1 <= nvec <= 256, tol > 0,
 *   maxit >= 1.  Returns
 *   KC_ERR_NO_CONVERGENCE after maxit iterations (c then holds the last iterate).  Op must be
 *   nonsingular: k = 0 is rejected only by the iteration failing to converge.
 */
int kc_pcg(kc_op* op, int ik, int nvec, const void* r, void* c, double tol, int maxit, int* iters, void* stream);

/*
 * kc_perturbed_residuals: training inputs from orthonormal vectors X [m][3][N^3] (converged
 *   eigenvectors of k-point ik): e = K_P^{-1} noise (eqs (2.31)-(2.32)), minus its orthogonal
 *   projection onto span(X), scaled to unit length; x_j = X_j + amp_j e_j; theta_j =
 *   <x_j, Op x_j> / <x_j, x_j> (Rayleigh quotient); r_j = Op x_j - theta_j x_j (FP64).
 *   noise: device [m][3][N^3]; amp: host double [m]; x (may be NULL) and r: device outputs
 *   [m][3][N^3], not overlapping X or noise.  1 <= m <= 32.
 */
int kc_perturbed_residuals(kc_op* op, int ik, int m, const void* X, const void* noise, const double* amp, void* x,
                           void* r, void* stream);

/*
 * kc_net_loss_grad: mean over j < nvec of the scale-free misfit of z_j = T_E r_j (E: the attached
 *   network's field for k-point ik, as kc_net_efield) against the targets c_j = Op^{-1} r_j:
 *   kind 0 (Op-norm, the norm of the eigensolver's convergence):
 *     min_alpha |alpha z - c|_Op^2 / |c|_Op^2 = 1 - (z^H r)^2 / ((z^H Op z)(c^H r));
 *   kind 1 (Euclidean): min_alpha |alpha z - c|^2 / |c|^2.
 *   *loss (host) receives the mean.  With gout != NULL (device float32 [N^3][16], the layout of
 *   the network's output y), also writes scale * d(mean)/dy: channels 0-2 through
 *   E = E0 exp(clamp(y, -3, 3)) (zero where the clamp is active), the other channels zero; the
 *   optimal alpha is held fixed (it is stationary).  1 <= nvec <= 256.  KC_ERR_INVALID_ARG when a
 *   c_j or T_E r_j is zero (the misfit is undefined).
 */
int kc_net_loss_grad(kc_op* op, int ik, int nvec, const void* r, const void* c, int kind, double scale, double* loss,
                     float* gout, void* stream);

/* Human-readable name of a status code. */
const char* kc_status_string(int status);

/* Message of the last error raised in this thread ("" if none). */
const char* kc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KCPC_H */
