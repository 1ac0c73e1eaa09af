/*
 * die_te.h -- C ABI of the MI355X (gfx950) solver for 2-D TE scattering by the
 * domain-integral-equation method of Zouros & Budko.
 *
 * Problem statement (Section 2 and Section 4 of the paper): an x3-invariant
 * object with relative permittivity eps_r(x) in a homogeneous background
 * (eps_b = mu_b = 1, no magnetic contrast) is illuminated by an incident
 * in-plane electric field E_in; the total field E = (E1, E2) solves
 *
 *     E_in = E - (k_b^2 + grad div) g * (chi E),  chi = eps_r - 1,
 *     g = (i/4) H0^(1)(k_b |x|)       (eqs. MatrixSolutionTE, GreenFunction)
 *
 * discretised by collocation with the midpoint rule on a uniform grid of square
 * cells (Section 4, eq. A11 and the element formulas that follow it):
 * A u = b with A = I - T X, X = diag(chi), T the Green tensor sampled at cell
 * separations (self cell integrated over the disc of equal area).
 *
 * Conventions shared by every entry point
 *   - Complex numbers are interleaved (re, im): complex128 = 2 doubles,
 *     complex64 = 2 floats (the layout of PyTorch complex tensors).
 *   - Field arrays are laid out [nrhs][ncomp][ny][nx], x fastest: ncomp = 2 for the TE
 *     E-block (component 0 = E1 = E_x, 1 = E2), 1 for TM (E3), 3 for the full TE system
 *     (E1, E2, H3) of die_te_setup_opts.magnetic; "2 nx ny" below reads ncomp nx ny.
 *     Cell (ix, iy) is centred at (x0 + (ix + 1/2) h, y0 + (iy + 1/2) h); only h enters
 *     the operator (it is translation invariant).
 *   - Units: lambda_b = 1 unless k_b says otherwise.
 *   - Pointers named "device" must point to GPU memory of the current device;
 *     the caller owns them and keeps them alive for the duration of the call
 *     (for asynchronous calls: until the stream reaches the call).  The
 *     library never frees or retains a caller pointer.
 *   - `stream` is a hipStream_t (NULL = the default stream).
 *   - Return codes: 0 = DIE_OK; > 0 = warning, outputs valid; < 0 = error,
 *     outputs unspecified, die_te_last_error() holds a message.  No entry point
 *     throws, aborts or exits.
 *   - A context is not thread safe: serialise calls that use it.
 */
#ifndef DIE_TE_H
#define DIE_TE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct die_te_ctx die_te_ctx;

enum {
  DIE_OK = 0,
  DIE_NOT_CONVERGED = 1, /* solve: tolerance not reached; the best iterate is returned */
  DIE_E_INVALID = -1,    /* bad argument (sizes, pointers, options) */
  DIE_E_SINGULAR = -2,   /* eps_r == 0 in some cell: existence condition eq. ExistenceTE fails */
  DIE_E_NOMEM = -3,      /* device or host allocation failed */
  DIE_E_HIP = -4,        /* a HIP runtime call failed */
  DIE_E_BREAKDOWN = -5   /* NaN/Inf met inside the Krylov iteration */
};

enum { DIE_C128 = 0, DIE_C64 = 1 }; /* precision of x and y for the operator products */

typedef struct {
  int nx, ny;   /* cells along x and y, each in [1, 2048] */
  double h;     /* cell side, > 0 */
  double k_b;   /* background wavenumber; 0 selects 2*pi (lambda_b = 1) */
  int px, py;   /* padded FFT grid; 0 selects the smallest power of two >= 2n-1
                   (any power of two >= 2n-1 and <= 4096 is accepted and gives
                   the same product: the linear convolution fits without wrap) */
} die_te_grid;

typedef struct {
  int regularize;          /* 1: solve A_R A u = A_R b with A_R = A(chi'), chi' = 1/eps_r - 1
                              (Section 3, eqs. InverseSymbol, Regularization; Section 5) */
  int deflate_k;           /* r >= 0: deflate the r largest-magnitude eigenvalues of the
                              solved operator (A_R A, or A) with the right preconditioner
                              P^-1 = I + V (T^-1 - I) V^*, T = V^* M V (Section 4,
                              eq. DeflatingPrecondtioner); 0 = no deflation;
                              -1 = automatic (Section 5): every eigenvalue beyond the
                              object's deflation radius (die_te_deflation_radius), r doubled
                              from 16 until fewer than r of the r largest Ritz values lie
                              beyond it, at most deflate_max; objects of one context may
                              then deflate different counts (die_te_deflation_info) */
  double eigs_tol;         /* Ritz pair accepted when ||M v - theta v|| <= eigs_tol |theta|; 0 -> 1e-4 */
  int eigs_krylov;         /* Krylov dimension of the eigensolver; 0 -> max(2r + 8, 24) */
  int eigs_max_restarts;   /* 0 -> 300 */
  unsigned long long seed; /* start vector of the eigensolver */
  int fft_variant;         /* 0: autotune the operator product's FFT passes (see
                              die_te_fft_plan); 1 + v: use variant v (0..3) in every pass */
  int deflate_max;         /* automatic deflation: largest r (0 -> 256; never above nx ny) */
  int polarization;        /* 0: TE (the default); 1: TM, the scalar operator of Section 2
                              eq. MatrixSolutionTM with chi_m = 0: E3_in = E3 - k^2 g * (chi E3),
                              collocated with the [A33] formulas of Section 4 (chi_e in place of
                              chi_m); fields have one component; no regularizer; automatic
                              deflation deflates outside the unit circle (Section 4, TM table) */
  int magnetic;            /* TE only.  1: the full system of Section 4 eq. lin_system on
                              u = (E1, E2, H3) with magnetic contrast chi_m = mu_r - 1: fields have
                              three components; the coupling blocks follow the compact kernels
                              K13, K23, K31, K32 of Section 3 (eps_b = mu_b = 1), A33 the [A33]
                              formulas; the regularizer, when on, uses chi' = 1/eps_r - 1 and
                              chi_m' = 1/mu_r - 1.  0: the E-block only (two components) */
  const void *mu_r;        /* magnetic = 1: device, complex128 [nobj][ny][nx] relative
                              permeability (copied at setup); NULL: mu_r = 1 (H3 is then computed
                              with the field, from E) */
} die_te_setup_opts;

typedef struct {
  int restart;       /* GMRES restart length m (>= 1, <= 510; the block solver: <= 65534 with
                        (m + 1) times the block width <= 65535) */
  int max_iters;     /* cap on the total number of inner GMRES iterations (>= 1) */
  double tol;        /* stop when ||b - A u||_2 <= tol ||b||_2, checked in FP64 on the
                        original (unregularized) operator; 0 -> 1e-8 */
  int mixed;         /* 0: FP64 throughout; 1: complex64 Krylov basis and operator products
                        inside an FP64 refinement loop (true residual, Hessenberg, Givens
                        and the deflation basis stay FP64); 2: as 1 with the Krylov basis
                        stored as complex binary16 (half the basis traffic; dots, Hessenberg
                        and Givens still FP64; needs orth = 1) */
  int x0_given;      /* 1: e_tot holds the initial guess on entry; 0: start from zero.  A
                        given guess whose FP64 residual ||b - A x0|| is non-finite or not
                        below ||b|| is replaced by zero (plain GMRES is the fallback) */
  double reg_margin; /* regularized runs end a cycle when the regularized residual estimate
                        reaches reg_margin * (the target scaled to the cycle); 0 -> 0.1 */
  int orth;          /* Arnoldi orthogonalisation: 0 = CGS2 (two projections per step, four
                        passes over the basis); 1 = CGS2 with the second projection of each
                        vector delayed to the next step (one block reduction and two passes
                        over the basis per step; equal in exact arithmetic) */
  int graph;         /* 1: capture the launches of one restart cycle's inner iterations once
                        into a HIP graph (on a stream the call creates) and replay it on
                        `stream` every cycle (fewer launches; the same results bit for bit);
                        0: launch them one by one.  Ignored while profiling is on. */
  int block;         /* 1: block GMRES(m): all right-hand sides of an object share one block
                        Krylov space (its first block spans their residuals, rank-revealed by a
                        pivoted Cholesky QR); CGS2 block orthogonalisation and CholQR2 of each
                        new block on the matrix cores (real products of planar copies of the
                        basis in the basis precision), the block least squares once per cycle
                        on the GPU; an object's right-hand sides run in groups of at most 64;
                        every cycle restarts from the FP64
                        true residual.  Needs mixed = 0 (FP64) or 1 (complex64 basis and
                        products).  orth = 0: two block Gram-Schmidt passes (CGS2); orth = 1:
                        one pass, the CholQR2 of the new block restoring its own
                        orthonormality.  graph does not apply.  iters counts block steps;
                        products_A per right-hand side is the object's share.
                        2: block GMRES as for 1 with mixed = 1 only, its block Gram-Schmidt
                        products Q^H W and W -= Q H on the binary16 matrix cores: a binary16
                        planar shadow of the basis (real and imaginary parts as separate real
                        columns) and of W, FP32 accumulation and FP32 W, the projection
                        coefficients rounded to binary16 (and kept so in H); CholQR, products
                        and least squares as for 1.
                        With mixed = 1 (block 1 or 2), a right-hand side whose full complex64
                        cycle reduces its FP64 true residual by less than 10% leaves the
                        complex64 iteration, and the call finishes it with FP64 block cycles
                        (its iters, products and cycles then count both phases).  When at most
                        16 right-hand sides of an object remain, a cycle's first block also
                        holds their corrections from the previous cycle.  The block solver
                        keeps its work buffers (and those corrections) in the context until
                        die_te_destroy.
                        0: per-rhs GMRES */
  int method;        /* 0: restarted GMRES (everything above).  1: Bi-CGSTAB; 2: restarted GCR(m) with
                        m = restart kept directions; 3: IDR(s) with s = restart <= 64 (a random
                        orthonormal shadow space from a fixed seed) (the Conclusions of the paper
                        name these as alternatives on the same preconditioned system): per right-hand side, in
                        FP64 (needs block = mixed = 0; orth and graph do not apply), on
                        M P^-1 v = A_R r exactly as GMRES; a right-hand side whose recurrence
                        residual reaches the tolerance scaled to the solved system, breaks down or
                        stagnates has its FP64 true residual checked and, if that is not below the
                        tolerance, restarts from it.  iters counts applications of M (two per
                        Bi-CGSTAB step); cycles counts true-residual checks */
} die_te_solve_opts;

typedef struct {
  int status;          /* DIE_OK or DIE_NOT_CONVERGED for this right-hand side */
  int iters;           /* inner GMRES iterations (each one applies the solved operator once) */
  int products_A;      /* applications of A (the FFT product), including residuals */
  int products_AR;     /* applications of A_R */
  int cycles;          /* GMRES cycles = FP64 residual refinements */
  double rel_res_true; /* final ||b - A u|| / ||b|| evaluated in FP64 */
  int finish_iters;    /* of iters, those run by the FP64 block cycles that finish a right-hand side
                          whose complex64 block cycles stalled (block = 2 or block = 1 with
                          mixed = 1); 0 otherwise */
} die_te_solve_info;

/* Build a context for one object: copies eps_r, evaluates the Green tensor on all
 * (2nx-1)(2ny-1) cell separations in FP64 on the host, embeds it circulantly in the
 * px x py grid, transforms it on the GPU once (the "symbol", shared by A and A_R,
 * as the paper notes for the regularizer) and, when deflate_k > 0, runs the
 * offline eigensolver.  eps_r: device, complex128 [ny][nx].  opts may be NULL
 * (defaults: no regularizer, no deflation).  Synchronises `stream`.
 * Returns DIE_E_SINGULAR if some eps_r is exactly 0. */
int die_te_setup(die_te_ctx **ctx, const die_te_grid *grid, const void *eps_r,
                 const die_te_setup_opts *opts, void *stream);

/* A context for nobj objects (1 <= nobj <= 65536) on one grid.  Each object is the
 * collocation system of Section 4 (eq. A11 family) on its own; the paper solves one
 * object and one incidence at a time, and solving many of them in the same launches
 * is this library's batching, not the paper's.  Every object shares the grid, hence
 * the symbol, and keeps its own contrasts and, when deflate_k > 0, its own deflation
 * data (one offline eigensolve per object; Section 4, eq. DeflatingPrecondtioner).
 * eps_r: device, complex128 [nobj][ny][nx].  Every entry point that takes nrhs
 * then requires nrhs to be a multiple of nobj and maps right-hand side r to
 * object r / (nrhs / nobj): fields are grouped object by object.  die_te_setup is
 * this call with nobj = 1.  Same return codes as die_te_setup. */
int die_te_setup_multi(die_te_ctx **ctx, const die_te_grid *grid, int nobj, const void *eps_r,
                       const die_te_setup_opts *opts, void *stream);

/* y = A x for nrhs fields (Section 4, eq. A11 family, realised by FFT convolution).
 * x, y: device, [nrhs][2][ny][nx] in the precision `prec` (DIE_C128 or DIE_C64);
 * x and y must not overlap.  Asynchronous on `stream`. */
int die_te_matvec(die_te_ctx *ctx, const void *x, void *y, int nrhs, int prec, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): y = A x exactly as die_te_matvec, with
 * the FFT intermediate (nrhs * 2 * px * ny4 complex values in the precision `prec`, ny4 = ny
 * rounded up to a multiple of 4) held
 * in a static per-device scratch array of 64 MiB instead of a buffer the context
 * allocates; the call allocates nothing and never tunes the FFT passes (it uses the
 * variants a die_te_matvec of the same batch-size class already uses, else the forced
 * variant, else the radix tuned for the grid).  DIE_E_INVALID when the intermediate
 * exceeds 64 MiB (e.g. 256 x 256 cells: at most 32 complex64 or 16 complex128 fields)
 * or when the context's device is not current.  Every call on one device shares that
 * device's array: calls that overlap in time on one device (different streams, or
 * threads) race and give wrong results; serialise them.  Same arguments otherwise as
 * die_te_matvec; asynchronous on `stream`. */
int die_te_matvec_noalloc(die_te_ctx *ctx, const void *x, void *y, int nrhs, int prec, void *stream);

/* y = A_R x = A(chi') x: the same operator with the regularizer contrast
 * chi' = 1/eps_r - 1 (Section 3, eq. InverseSymbol; Section 5).  Same arguments
 * and semantics as die_te_matvec. */
int die_te_regularize(die_te_ctx *ctx, const void *x, void *y, int nrhs, int prec, void *stream);

/* Solve A u = b for nrhs incident fields with restarted GMRES (Section 4) on
 * M P^-1 v = A_R r  (M = A_R A when regularized, else A; P^-1 the deflation
 * preconditioner when the context has one; u += P^-1 v), each cycle restarted
 * from the FP64 true residual r = b - A u.  All right-hand sides advance
 * together in batched kernels; each stops on its own.
 * e_in:  device, complex128 [nrhs][2][ny][nx], the sampled incident field b.
 * e_tot: device, complex128, same shape: the total field u (initial guess on
 *        entry when opts->x0_given).
 * info:  host array of nrhs records (may be NULL).
 * Returns DIE_OK when every RHS converged, DIE_NOT_CONVERGED when some did not
 * (each of those gets back the iterate with the lowest FP64 true residual met at the
 * start of a cycle, and info reports that residual), < 0 on error (info records the
 * solver did not reach read status < 0).  Synchronises `stream`. */
int die_te_solve(die_te_ctx *ctx, const void *e_in, void *e_tot, int nrhs,
                 const die_te_solve_opts *opts, die_te_solve_info *info, void *stream);

/* Objects on grids of different sizes in one call (the same solver as die_te_solve,
 * Section 4): context i (one grid size, one or more objects) solves nrhs[i] incident
 * fields e_in[i] -> e_tot[i] (each laid out as in die_te_solve for that context) with the
 * shared options; info[i] receives nrhs[i] records (info, or any info[i], may be NULL).
 * Work queued on `stream` before the call completes first; the contexts then advance
 * concurrently, each on a stream of its own that the call creates (default priority) and
 * destroys, and the call returns when all have finished.  The contexts must be distinct.
 * Returns the first error (< 0, in context order; die_te_last_error() names the context),
 * else DIE_NOT_CONVERGED if any right-hand side did not converge, else DIE_OK. */
int die_te_solve_batch(die_te_ctx *const *ctx, int nctx, const void *const *e_in, void *const *e_tot,
                       const int *nrhs, const die_te_solve_opts *opts, die_te_solve_info *const *info,
                       void *stream);

/* The dense matrix of one of the context's operators for object obj (the spectral analysis of
 * Sections 4 and 5, Figs. 2 and 3): which = 0 A, 1 A_R, 2 A_R A, 3 the operator GMRES solves
 * (M P^-1: M = A_R A when the context is regularized, else A; P^-1 the deflation preconditioner
 * when it has one).  Column j is the operator applied to the unit vector e_j in FP64 (batches
 * of identity columns through the FFT products).  out: device, complex128, nvec x nvec
 * column-major (nvec = ncomp nx ny), owned by the caller.  Synchronises `stream`. */
int die_te_operator_dense(die_te_ctx *ctx, int which, int obj, void *out, void *stream);

/* All eigenvalues of that matrix (same which and obj), for nvec <= 4096 (DIE_E_INVALID above):
 * the dense matrix is formed on the GPU as above and reduced on the host (Householder
 * Hessenberg reduction and shifted QR, O(nvec^3)).  eig: host, nvec complex128 values (order of
 * the Schur form's diagonal).  DIE_E_BREAKDOWN if the QR iteration does not converge.
 * Synchronises `stream`. */
int die_te_spectrum(die_te_ctx *ctx, int which, int obj, void *eig, void *stream);

/* P^-1 x = x + V ((T^-1 - I) (V^* x)) for nrhs complex128 vectors of length 2 nx ny
 * (Section 4, eq. DeflatingPrecondtioner).  x, y: device; may alias.
 * DIE_E_INVALID if the context has no deflation basis.  Asynchronous. */
int die_te_apply_deflation(die_te_ctx *ctx, const void *x, void *y, int nrhs, void *stream);

/* Read back the deflation data: r (host int), the r Ritz values of largest
 * magnitude (host complex128 [nobj][r], may be NULL), the orthonormal bases V
 * (device complex128 [nobj][r][2][ny][nx], may be NULL) and C = T^-1 - I (host
 * complex128 [nobj][r][r] row-major, may be NULL).  An object whose Krylov space
 * closes before r vectors has zero rows in V and C past its last vector, which
 * leaves its P^-1 unchanged there.  Synchronises `stream`. */
int die_te_deflation_info(die_te_ctx *ctx, int *r, void *ritz_values, void *V, void *C,
                          void *stream);

/* The FFT pass variants the operator products of nrhs fields in precision `prec` use:
 * variants[0..2] for the row transform, the column transform with the symbol multiply and
 * the inverse row transform.  Variant v: bit 0 set takes the other register radix (8 <->
 * 16), bit 1 set halves the tile (rows or columns per block); only transforms of length
 * >= 128 have variants.  Unless the context forces a variant (fft_variant at setup), the
 * library picks them by timing the variants on the context's grid the first time a
 * product of that precision and batch-size class (1-2, 3-32, > 32 fields) runs, or here:
 * the radix of each pass once per device, precision and grid shape for the whole process
 * (it changes the rounding, so every context and batch shares it), the tile per batch-size
 * class (results are equal bit for bit).  Tuning allocates scratch for min(nrhs, 64)
 * fields and synchronises `stream`. */
int die_te_fft_plan(die_te_ctx *ctx, int prec, int nrhs, int *variants, void *stream);

/* Diagnostic: in-place unnormalised forward (inverse = 0) or backward
 * (inverse = 1, also unnormalised) 2-D FFT of `batch` complex arrays
 * [batch][py][px] with the library's own FFT kernels; px, py powers of two in
 * [2, 4096].  data: device, complex128 (prec = DIE_C128) or complex64.
 * Synchronises `stream`. */
int die_te_fft2(void *data, int px, int py, int batch, int inverse, int prec, void *stream);

/* Diagnostic timing.  die_te_profile(ctx, s) with s >= 1 clears the counters and starts
 * bracketing, with hipEvents on the stream each launch is issued on, one in every s
 * launches of each kind: operator products (the three FFT passes of one application of
 * A or A_R: kind DIE_PROF_PRODUCT), Arnoldi dot-product kernels (DIE_PROF_DOTS),
 * Arnoldi multi-axpy kernels (DIE_PROF_AXPY) and the block solver's basis-update GEMMs
 * W -= Q H (DIE_PROF_GEMM) issued through the context;
 * die_te_profile(ctx, 0) stops.
 * die_te_profile_read returns the number of bracketed launches of `kind`, the number of
 * launches of that kind issued while profiling was on (`seen`, may be NULL), the total
 * elapsed milliseconds of the bracketed ones (synchronises on the recorded events) and
 * (`bytes`, may be NULL) the sum of their algorithmic HBM bytes: the compulsory reads and
 * writes of each launch's operands for the right-hand sides live when it was issued
 * (inside a solve: those active at the start of the GMRES cycle).  Products:
 * es (2RN + n_obj N + 8R ny px + 3 px py + 4RN) with es the bytes per complex value;
 * dots over j basis vectors: R (j + 1) 2N es; multi-axpys: R (j + 2) 2N es.  For
 * DIE_PROF_GEMM the `bytes` output holds flops instead: 8 M N K per complex GEMM.
 * die_te_profile_mem returns in *mem_bytes the algorithmic HBM bytes of the bracketed
 * launches of `kind` (the same figure as `bytes` for the first three kinds; for
 * DIE_PROF_GEMM the operand bytes es (n nq + 2 n p + nq p) of each update W -= Q H with
 * W of n x p and Q of n x nq).  DIE_E_INVALID for a bad kind or a NULL output. */
enum { DIE_PROF_PRODUCT = 0, DIE_PROF_DOTS = 1, DIE_PROF_AXPY = 2, DIE_PROF_GEMM = 3 };
int die_te_profile(die_te_ctx *ctx, int enable);
int die_te_profile_read(die_te_ctx *ctx, int kind, long long *launches, long long *seen, double *total_ms,
                        double *bytes);
int die_te_profile_mem(die_te_ctx *ctx, int kind, double *mem_bytes);

/* Section 5's deflation radius R of an object: the dense segment [1, eps(x)] of the
 * spectrum of A at every cell mapped through eq. EigenvaluesArA (regularized != 0, the
 * solved operator A_R A) or taken as it is (regularized == 0, A), the largest magnitude over
 * all cells: R = max_x max(1, |1 + (eps - 1)^2 / (4 eps)|) or max_x max(1, |eps|).
 * eps_r: HOST complex128 [ncells].  DIE_E_SINGULAR if some eps_r is 0.  No GPU work. */
int die_te_deflation_radius(const void *eps_r, long long ncells, int regularized, double *radius);

/* The memory planner of Section 5 (its systematic application, steps 1-5) for the paper's
 * 3N-unknown system with 16-byte complex values: a memory budget of mem_bytes, the ratio
 * beta = r / (3N) of deflated eigenvalues, a grid of points_per_wavelength points per
 * smallest medium wavelength, restart = x r and the largest real relative permittivity.
 * The grid follows from M_A + M_prec = mem_bytes with M_A = 720 N and
 * M_prec = 16 r^2 + 48 N r + 48 N restart; the unpreconditioned system gets restart + r
 * (the same memory).  This library's TE solver keeps 2N unknowns, 2/3 of the vectors
 * counted here.  No GPU work. */
typedef struct {
  double alpha;              /* points_per_wavelength * sqrt(eps_re_max) */
  double n_max;              /* the largest affordable number of grid points */
  double a_over_lambda_max;  /* the largest affordable object size (sqrt(n_max) - 1) / alpha */
  long long nodes;           /* grid points per side of that object, floor(sqrt(n_max)) */
  long long n;               /* nodes^2 */
  long long unknowns;        /* 3 n */
  int r;                     /* deflated eigenvalues, ceil(3 n beta) */
  int restart;               /* restart of the preconditioned system, x r */
  int restart_unpreconditioned; /* restart + r */
  double mem_system;         /* M_A, bytes */
  double mem_preconditioner; /* M_prec, bytes */
} die_te_plan;
int die_te_plan_memory(double mem_bytes, double beta, double points_per_wavelength, double x, double eps_re_max,
                       die_te_plan *plan);

/* Release everything the context owns. */
int die_te_destroy(die_te_ctx *ctx);

/* Message for the most recent error return in the calling thread ("" if none). */
const char *die_te_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DIE_TE_H */
