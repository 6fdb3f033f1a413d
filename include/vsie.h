/*
 * vsie.h -- C ABI of libvsie.so, the MI355X (gfx950) implementation of the
 * discretised nested volume-surface integral equation (VSIE) for acoustics.
 *
 * The operator is the collocation form of the final VSIE (Theorem 3, eq_vsie,
 * of "Nested Volume-Surface Integral Equations for Acoustics"):
 *
 *     (A p)_i = m_i p_i - (V p)_i + (T p)_i + (K p)_i
 *
 * over the unknowns (p_Omega1, p_Omega2, p_Gamma1, p_Gamma2) of the 4x4 block
 * system (section 2.3.4), with P0 elements, collocation at element centroids,
 * the one-point (midpoint) rule for every off-diagonal integral and the
 * weakly singular self-term of V integrated on the sphere of equal volume
 * (section 2.3.5).  For i != j:
 *
 *     A_ij = -G(r_ij) s_j + F(r_ij) (x_i - y_j) . v_j,
 *     G(r) = exp(i k0 r) / (4 pi r),    F(r) = exp(i k0 r)(i k0 r - 1) / (4 pi r^3)
 *
 * volume cell j : s_j = |cell| (beta - k0^2 alpha)(y_j)   (eq_alpha, eq_beta)
 *                 v_j = |cell| grad alpha(y_j)
 * surface elt j : s_j = 0,  v_j = -|face| (alpha_inside - alpha_outside) n_j
 * diagonal      : A_ii = m_i - (s_i/|cell_i|) S(a_i, k0) on cells (eq_mass_function
 *                 for m; S = integral of G over the ball of radius a_i of equal
 *                 volume), A_ii = m_i on surface elements.
 *
 * Conventions for every call
 * --------------------------
 * * Complex vectors live in device memory as interleaved (re, im) doubles
 *   (complex128), column-major n x nrhs with a leading dimension counted in
 *   complex elements (ld >= n).  Unknown order: volume cells in the caller's
 *   order, then surface elements in the caller's order (callers pass Omega_1
 *   then Omega_2, Gamma_1 then Gamma_2, the paper's block order).
 * * `stream` is a hipStream_t (NULL selects the null stream).  Calls enqueue
 *   work on it; vsie_solve synchronises it to read scalars each iteration.
 *   When a product returns an error, work it queued before the error may
 *   still run on `stream`; the solves synchronise `stream` before returning,
 *   also on error.
 * * No exception crosses the ABI: every call returns a vsie_status, and
 *   vsie_last_error() gives a message for the calling thread's last failure.
 * * Memory: input host arrays are copied during vsie_assemble; the problem
 *   owns its device arrays (geometry, weights) until vsie_destroy.  Vectors
 *   x, y, b are owned by the caller.  Work buffers (partial sums, packed
 *   charges, Krylov bases) come from the caller's workspace when the call is
 *   given one (`workspace`, `ws_bytes`: DEVICE memory, 256-byte aligned, at
 *   least vsie_workspace_size bytes, not touched by anything else while the
 *   call's work runs on `stream`); with workspace == NULL the problem keeps
 *   its own grow-only buffers, reused by later calls (growing one waits for
 *   the whole device, because kernels queued on any stream may still read
 *   the old buffer).  A call given a workspace allocates no device memory
 *   for work buffers.
 * * A problem handle may be used from one host thread at a time.
 */
#ifndef VSIE_H
#define VSIE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VSIE_OK = 0,
    VSIE_E_INVALID = 1,   /* bad argument: NULL pointer, size, index, material, normal */
    VSIE_E_DEVICE = 2,    /* a HIP runtime call failed */
    VSIE_E_NOMEM = 3,     /* device allocation failed */
    VSIE_E_NOCONV = 4,    /* solver stopped at max_iter; x holds the last iterate */
    VSIE_E_NAN = 5,       /* a non-finite value appeared in a residual norm */
    VSIE_E_WORKSPACE = 6  /* the caller's workspace is smaller than the call needs */
} vsie_status;

/* Arithmetic of the operator.
 * VSIE_FP64: every pair term in FP64.
 * VSIE_FP32: pair terms and their sums over a tile of sources in FP32, with
 *   target-source distances and the phase k0 r reduced in FP64, tile sums
 *   gathered in FP64; the diagonal (mass function and self-terms) stays FP64.
 *   In vsie_solve this selects FP32 GMRES inner solves inside FP64 iterative
 *   refinement (residuals b - A x with the FP64 operator). */
typedef enum { VSIE_FP64 = 0, VSIE_FP32 = 1 } vsie_precision;

typedef struct vsie_problem vsie_problem;

/* Mesh of the nested domains (section 2.3.1: cuboid cells, surface elements
 * that match cell faces).  All arrays are host memory, read during
 * vsie_assemble only. */
typedef struct {
    int64_t n_vol;                  /* number of volume cells (>= 0) */
    const double *vx, *vy, *vz;     /* cell centroids */
    const double *vw;               /* cell volumes (> 0) */
    const int32_t *vdom;            /* subdomain of each cell: 1 or 2 */
    const int32_t *vnb;             /* 6*n_vol face neighbours (-x,+x,-y,+y,-z,+z),
                                       -1 for none; NULL means no neighbours */
    const double *vgrad_alpha;      /* optional 3*n_vol (x,y,z per cell) grad alpha
                                       overriding the neighbour stencil; or NULL */
    const double *vgrad_rho;        /* optional 3*n_vol (x,y,z per cell) gradient of an
                                       analytic density at the centroids: grad alpha =
                                       -rho0 grad(rho) / rho^2 (eq_alpha), used when
                                       vgrad_alpha is NULL, instead of the stencil; or NULL */
    int64_t n_srf;                  /* number of surface elements (>= 0) */
    const double *sx, *sy, *sz;     /* element centroids */
    const double *snx, *sny, *snz;  /* unit normals pointing out of the inside
                                       subdomain (|n| = 1 within 1e-12) */
    const double *sarea;            /* element areas (> 0) */
    const int32_t *siface;          /* 1 (Gamma_1) or 2 (Gamma_2) */
    const int32_t *scell_in;        /* cell on the inside of the face */
    const int32_t *scell_out;       /* cell on the outside, -1 = exterior Omega_0 */
    double rho0, c0;                /* exterior density and speed of sound (> 0) */
} vsie_geometry;

/* Build a problem: validate and upload the mesh and the per-cell materials,
 * and compute the per-element weights for n_freq exterior wavenumbers k0[f]
 * (omega_f = k0[f] c0).
 *   vrho, vc : host arrays of n_vol cell densities and sound speeds (> 0).
 * Interface limit densities are those of the cells on either side of a face.
 * grad alpha (when vgrad_alpha is NULL) is a per-axis central difference of
 * alpha = rho0/rho - 1 over the face neighbours in the same subdomain,
 * one-sided with one such neighbour and zero with none.
 * On success *out receives a new handle; on failure *out is NULL. */
vsie_status vsie_assemble(const vsie_geometry *geom, const double *vrho, const double *vc,
                          const double *k0, int32_t n_freq, void *stream, vsie_problem **out);

/* Replace the per-cell materials from DEVICE arrays (n_vol doubles each) and
 * recompute every weight (used between solves of an optimisation loop).  The
 * set of nonzero source terms may change; the call synchronises `stream`.
 * Materials that are not positive and finite are rejected with VSIE_E_INVALID
 * before anything is written: the problem keeps its previous materials,
 * weights and sources. */
vsie_status vsie_set_materials(vsie_problem *p, const double *vrho_dev, const double *vc_dev,
                               void *stream);

/* Number of unknowns n = n_vol + n_srf (0 for a NULL handle). */
int64_t vsie_size(const vsie_problem *p);

/* Number of volume cells n_vol (the length of the material arrays of
 * vsie_set_materials and of the gradients of vsie_param_gradient; 0 for a
 * NULL handle). */
int64_t vsie_num_cells(const vsie_problem *p);

/* y = A_f x for nrhs right-hand sides at frequency index f.
 * x, y: device complex128, n x nrhs, leading dimensions ldx, ldy; x and y
 * must not overlap.  workspace, ws_bytes: optional caller workspace (see the
 * conventions above; NULL, 0 for the problem's own buffers); too small gives
 * VSIE_E_WORKSPACE before any work is queued. */
vsie_status vsie_matvec(vsie_problem *p, int32_t f, vsie_precision prec, int64_t nrhs,
                        const double *x, int64_t ldx, double *y, int64_t ldy, void *workspace,
                        size_t ws_bytes, void *stream);

/* y = A_f^H x (conjugate transpose), same layout and workspace rules as
 * vsie_matvec. */
vsie_status vsie_matvec_adjoint(vsie_problem *p, int32_t f, vsie_precision prec, int64_t nrhs,
                                const double *x, int64_t ldx, double *y, int64_t ldy,
                                void *workspace, size_t ws_bytes, void *stream);

/* y_t = A_{f0+t} x_t for the nf frequencies f0 .. f0 + nf - 1 at once: x and
 * y hold nf consecutive blocks of nrhs columns, block t (frequency f0 + t)
 * starting at column t nrhs (same layout rules as vsie_matvec).  With
 * VSIE_FP32 and nrhs >= the tuning's mfma_min_rhs, each source class runs in
 * one matrix-core launch over all nf frequencies; otherwise the
 * frequencies are applied one after the other. */
vsie_status vsie_matvec_multi(vsie_problem *p, int32_t f0, int32_t nf, vsie_precision prec, int64_t nrhs,
                              const double *x, int64_t ldx, double *y, int64_t ldy, void *workspace,
                              size_t ws_bytes, void *stream);


/* Launch configuration of the pair products of one problem.
 *
 * FP32 forward products (vsie_matvec, vsie_matvec_multi, the inner solves of
 * vsie_solve) with at least mfma_min_rhs right-hand sides evaluate each pair
 * kernel once on the vector ALUs and apply it to 16-column blocks of
 * right-hand sides on the matrix cores (v_mfma_f32_16x16x4_f32, FP32
 * accumulation over tiles of 128 sources, then FP64), in one launch whose
 * work items are (frequency, column block, source chunk, target tile), one
 * item per wave.
 * Other products use the vector pair kernel, one thread per target. */
typedef struct {
    int32_t mfma_min_rhs;      /* 0 = never use the matrix cores; default 8 */
    int32_t mfma_tg;           /* 16-target groups per wave: 2 or 4; default 2 */
    int32_t mfma_nb;           /* 16-column blocks per work item: 1 or 2; default 1 */
    int32_t items_per_wave;    /* matrix-core work items per wave the chip holds at
                                  once, which sets the source chunk length (>= 1);
                                  default 16 */
    int64_t vec_target_waves;  /* waves per vector pair launch, which sets its source
                                  chunk length (>= 1024); default 32768 */
    int32_t graph;             /* 1: inside vsie_solve, each operator application of
                                  the matrix-free paths (pack, pair and reduction
                                  launches) is captured once into a hipGraph and
                                  replayed every iteration; 0: launched one by one;
                                  default 1 */
    int32_t sym_groups;        /* one-column forward products: when every cell is a
                                  single-layer source, the cell-cell single layer runs
                                  once per unordered pair (e_ij = e_ji), in work items
                                  of sym_groups x sym_groups 64-cell tiles; 0 = off,
                                  2, 4 or 8; default 4.  Each cell keeps one partial
                                  sum per partner group: the group size is doubled
                                  (up to 8) while these would exceed 8 GiB at the
                                  FP64 size, and above 64 GiB the one-sided kernels
                                  run instead */
    int32_t cell_face;         /* with sym_groups on: the cell-face pairs also run
                                  once per pair (single layer and adjoint double
                                  layer of the cell at the face, double layer of the
                                  face at the cell), the cells' adjoint double layers
                                  (grad alpha) ride along the cell-cell single
                                  layer, and only the faces with a double-layer
                                  weight are summed over the faces one-sided;
                                  0 = off, 1 = on; default 1 */
    int32_t mfma_3m;           /* matrix-core products: 0 = four real products per
                                  complex multiply-add (Kr Qr, Ki Qi, Kr Qi, Ki Qr),
                                  1 = three (Kr Qr, Ki Qi, (Kr + Ki)(Qr + Qi); the
                                  imaginary part as the difference of FP32 sums);
                                  default 1; the FP64 matrix-core products follow
                                  the same choice */
    int32_t mfma64_min_rhs;    /* FP64 forward products (vsie_matvec, vsie_matvec_multi,
                                  the FP64 products and residuals of vsie_solve) with at
                                  least this many right-hand sides evaluate each pair
                                  kernel once in FP64 on the vector ALUs and apply it to
                                  16, 32 or 64 columns on the FP64 matrix cores
                                  (v_mfma_f64_16x16x4_f64, FP64 accumulation); 0 = never;
                                  default 16 */
    int32_t mfma_chunk_max;    /* matrix-core products (FP32 and FP64): at most this many
                                  sources per chunk, 0 = no cap (>= 1024 otherwise).
                                  The waves of one XCD walk the target tiles of one
                                  chunk, so a cap keeps the source positions and charges
                                  they stream within the last-level cache on large
                                  problems; every chunk adds one FP64 partial per
                                  target and column (frequencies x columns x n x 16
                                  bytes per chunk) */
} vsie_tuning;

vsie_status vsie_get_tuning(const vsie_problem *p, vsie_tuning *out);
/* Rejects values outside the ranges above (VSIE_E_INVALID, tuning unchanged). */
vsie_status vsie_set_tuning(vsie_problem *p, const vsie_tuning *t);

/* Autotuner: times every candidate configuration of the FP32 forward product
 * with nrhs right-hand sides at frequency f (the vector kernel at three chunk
 * lengths; the matrix-core kernel at each (mfma_tg, mfma_nb) and three
 * items_per_wave when nrhs >= 8), two launches each after a warm-up, keeps the
 * fastest in the problem's tuning and copies it to *best (may be NULL).
 * Allocates and frees its own input and output blocks; synchronises stream. */
vsie_status vsie_autotune(vsie_problem *p, int32_t f, int64_t nrhs, vsie_tuning *best, void *stream);

typedef struct {
    double tol;          /* stop when ||b - A x|| <= tol ||b|| (FP64 residual); default 1e-10 */
    int32_t max_iter;    /* total GMRES iterations (all cycles, all outer steps); default 3000 */
    int32_t restart;     /* Krylov dimension per cycle; default 500, lowered when the
                            basis of all nrhs right-hand sides would exceed half of the
                            Krylov budget (krylov_gib: two bases of half of it each, the
                            first cycle's kept to deflate the later cycles) */
    double inner_tol;    /* VSIE_FP32 only: relative tolerance of each inner solve; default 1e-5 */
    int32_t max_outer;   /* VSIE_FP32 only: refinement steps; default 20 */
    int32_t block;       /* 0: an independent GMRES per right-hand side, advanced in
                            lockstep (later cycles deflated by the first cycle's space);
                            1: block GMRES -- one block Krylov space for all right-hand
                            sides of a cycle, restart counted in block steps and capped
                            so that (steps x nrhs) <= 11585; default 0 */
    double relax;        /* VSIE_FP32 with block = 0 only.  0: iterative refinement, every
                            GMRES iteration with the FP32 operator (default).  > 0: relaxed
                            products -- each cycle aims at the final tolerance and an
                            iteration applies the FP64 operator while the cycle's residual
                            estimate exceeds (cycle tolerance / relax) x its starting
                            residual, the FP32 operator after that.  relax is the relative
                            error assumed for an FP32 product (e.g. 1e-6): a product may be
                            that inexact once the residual has fallen far enough that its
                            error can no longer lift the final residual above the
                            tolerance (inexact Krylov methods). */
    int32_t progress;    /* 1: one line on stderr per outer step (FP64 residual), per block
                            step and every 25 GMRES iterations (residual estimate), for long
                            solves; 0: silent (default) */
    int32_t krylov_gib;  /* device memory of the two Krylov bases together, in GiB (half
                            each); it caps the restart length as described under restart.
                            0: 96 (default), which leaves room for an assembled operator;
                            at most 4096.  A large problem without an assembled operator
                            (and a multi-frequency solve, whose frequencies share it) may
                            raise it toward the free device memory. */
} vsie_solve_opts;

typedef struct {
    int32_t iterations;     /* GMRES iterations summed over right-hand sides */
    int32_t outer_steps;    /* most GMRES cycles of any right-hand side (refinement steps
                               for VSIE_FP32, restart cycles for VSIE_FP64) */
    int32_t matvecs_fp64;   /* single-column operator applications in FP64, summed over
                               right-hand sides */
    int32_t matvecs_fp32;   /* the same in FP32 */
    double rel_residual;    /* max over right-hand sides of ||b - A x|| / ||b|| */
} vsie_solve_info;

/* Solve A_f x = b (adjoint = 0) or A_f^H x = b (adjoint = 1) by GMRES without
 * preconditioning (section 3.1), restarted every opts->restart iterations.
 * The nrhs right-hand sides run independent GMRES processes in lockstep: each
 * iteration applies the operator to all unconverged columns in one launch.
 * x holds the initial guess on entry and the solution on exit.  opts may be
 * NULL (defaults); info may be NULL.  nrhs <= 4096.  workspace, ws_bytes: as
 * for vsie_matvec (bases, residual blocks and the operator's buffers; block
 * GMRES's rocBLAS handle keeps device memory of its own).  Returns
 * VSIE_E_NOCONV when the tolerance was not reached (x still holds the last
 * iterate). */
vsie_status vsie_solve(vsie_problem *p, int32_t f, vsie_precision prec, int32_t adjoint,
                       int64_t nrhs, const double *b, int64_t ldb, double *x, int64_t ldx,
                       const vsie_solve_opts *opts, vsie_solve_info *info, void *workspace, size_t ws_bytes,
                       void *stream);

/* Solve A_f x = b for the nf frequencies f = f0 .. f0 + nf - 1 of one
 * problem together (forward operator; the scattering problem of section 3.1 at
 * several wavenumbers).  Layout as vsie_matvec_multi: frequency f0 + t owns
 * columns t nrhs .. (t + 1) nrhs - 1 of b and x (leading dimensions ldb,
 * ldx >= n).  Each frequency runs its own block GMRES -- for VSIE_FP32 inside
 * FP64 iterative refinement -- exactly as vsie_solve with opts->block = 1
 * would, except for the restart length; the processes advance in lockstep and
 * share the operator launches: every block step applies the operators of all
 * frequencies still iterating as one multi-frequency launch per source class
 * (one per run of consecutive frequencies of equal block width; widths below
 * the matrix-core thresholds of vsie_tuning fall back to one product per
 * frequency), and every FP64 refinement residual likewise.  A frequency whose
 * cycle has ended waits for the others before its next refinement step.  The
 * nf bases share the Krylov budget of one solve, so a frequency's cycle is
 * capped at the block steps a single solve of nf nrhs columns would get.
 * opts->block and opts->relax are ignored; opts->tol, max_iter, restart,
 * inner_tol, max_outer and progress apply to every frequency.  info: NULL or
 * an array of nf entries, one per frequency.  nrhs <= 4096.  workspace,
 * ws_bytes: as for vsie_solve (VSIE_OP_SOLVE_MULTI).  Returns VSIE_E_NOCONV
 * when any frequency missed the tolerance (its x holds the last iterate). */
vsie_status vsie_solve_multi(vsie_problem *p, int32_t f0, int32_t nf, vsie_precision prec, int64_t nrhs,
                             const double *b, int64_t ldb, double *x, int64_t ldx, const vsie_solve_opts *opts,
                             vsie_solve_info *info, void *workspace, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): y = A_f x
 * exactly as vsie_matvec computes it (same kernels, same results), with its
 * work buffers in a static device work area of the library instead of
 * problem-owned or caller memory.  The area holds 256 MiB (268,435,456
 * bytes) per GPU, is created with the library's code object on each device
 * it runs on and held until the process ends; its device address is looked
 * up once per device on the first call there.  A product whose work buffers
 * (vsie_workspace_size with VSIE_OP_MATVEC) exceed it is refused with
 * VSIE_E_WORKSPACE before anything is written.  The call allocates no device
 * memory and records no profiler events.  The problem's device must
 * be current.  All calls on one GPU share its area: calls that overlap in
 * time (other streams, other threads, other problems) race; calls ordered
 * on one stream do not, and nothing in the area needs clearing between
 * them. */
vsie_status vsie_matvec_noalloc(vsie_problem *p, int32_t f, vsie_precision prec, int64_t nrhs,
                                const double *x, int64_t ldx, double *y, int64_t ldy, void *stream);

/* The calls that take a caller workspace. */
typedef enum {
    VSIE_OP_MATVEC = 0,          /* vsie_matvec */
    VSIE_OP_MATVEC_ADJOINT = 1,  /* vsie_matvec_adjoint */
    VSIE_OP_MATVEC_MULTI = 2,    /* vsie_matvec_multi over nf frequencies from f */
    VSIE_OP_SOLVE = 3,           /* vsie_solve, adjoint = 0 */
    VSIE_OP_SOLVE_ADJOINT = 4,   /* vsie_solve, adjoint = 1 */
    VSIE_OP_SOLVE_MULTI = 5      /* vsie_solve_multi over nf frequencies from f */
} vsie_op;

/* Bytes of workspace the call `op` needs on problem p for frequency f (nf
 * frequencies for VSIE_OP_MATVEC_MULTI and VSIE_OP_SOLVE_MULTI, else 1), precision prec and nrhs
 * right-hand sides, with solver options opts (solves only; NULL = defaults)
 * and the problem's current tuning, materials and assembled operators.  A
 * change of any of these may change the size.  Writes *bytes. */
vsie_status vsie_workspace_size(vsie_problem *p, vsie_op op, int32_t f, int32_t nf, vsie_precision prec,
                                int64_t nrhs, const vsie_solve_opts *opts, size_t *bytes);

/* b[:, r] = exp(i k0_f x_i . d_r) at every collocation point for ndir unit
 * directions given as a HOST array of 3*ndir doubles (eq_planewave). */
vsie_status vsie_plane_wave(vsie_problem *p, int32_t f, int64_t ndir, const double *dirs,
                            double *b, int64_t ldb, void *stream);

/* out[t, r] = sum_j A_f(x_t, j) x[j, r] at n_t arbitrary target points given
 * as DEVICE arrays tx, ty, tz (the off-diagonal kernel with no self term).
 * The exterior field of section 2.3.1 is p(x) = p_inc(x) - out. */
vsie_status vsie_field(vsie_problem *p, int32_t f, vsie_precision prec, int64_t n_t,
                       const double *tx, const double *ty, const double *tz, int64_t nrhs,
                       const double *x, int64_t ldx, double *out, int64_t ldo, void *stream);

/* Far-field pattern of the scattered pressure: the exterior field of section
 * 2.3.1 along a unit direction d as |x| = R -> infinity,
 *   p(R d) - p_inc(R d) = exp(i k0 R)/R pinf(d) + O(R^-2),
 *   pinf(d) = 1/(4 pi) sum_j exp(-i k0 d.y_j) (s_j - i k0 d.v_j) x[j, r]
 * (s_j, v_j the single-layer and double-layer weights of element j, see the
 * top of this file; G and grad G replaced by their leading terms).
 *   dx, dy, dz : n_d DEVICE doubles, the directions (unit length, not checked)
 *   x          : n x nrhs DEVICE solution columns, ldx >= n
 *   out        : n_d x nrhs DEVICE, out[t + r ldo] = pinf(d_t) of column r, ldo >= n_d
 * FP32 evaluates the amplitudes in FP32 (phase k0 d.y formed and reduced in
 * FP64) and adds FP32 sums of at most 128 sources in FP64. */
vsie_status vsie_far_field(vsie_problem *p, int32_t f, vsie_precision prec, int64_t n_d,
                           const double *dx, const double *dy, const double *dz, int64_t nrhs,
                           const double *x, int64_t ldx, double *out, int64_t ldo, void *stream);

/* Source-side sums for adjoint-state gradients:
 *   z[j, r]      = sum_t conj(G(|x_t - y_j|)) lam[t, r]
 *   Z[j, r, a]   = sum_t conj(F(|x_t - y_j|)) (x_t - y_j)_a lam[t, r]
 * Targets are the collocation points themselves (t != j) when tx is NULL
 * (n_t must then equal n), otherwise n_t DEVICE points.  z: n x nrhs,
 * ldz >= n; Z: n x (3 nrhs), column 3 r + a, ldZ >= n. */
vsie_status vsie_source_sums(vsie_problem *p, int32_t f, int64_t n_t, const double *tx,
                             const double *ty, const double *tz, int64_t nrhs,
                             const double *lam, int64_t ldl, double *z, int64_t ldz, double *Z,
                             int64_t ldZ, void *stream);

/* b[:, r] = exp(i k0_f t . d_r) at n_t DEVICE points (tx, ty, tz), for ndir
 * unit directions given as a HOST array of 3*ndir doubles (eq_planewave). */
vsie_status vsie_plane_wave_at(vsie_problem *p, int32_t f, int64_t ndir, const double *dirs,
                               int64_t n_t, const double *tx, const double *ty, const double *tz,
                               double *out, int64_t ldo, void *stream);

/* Right-hand side of the adjoint system of a receiver misfit:
 *   out[j, r] = s_j zR[j, r] - v_j . ZR[j, r]
 * (s_j, v_j the single-layer and double-layer weights of element j, see the
 * top of this file; zR, ZR from vsie_source_sums over the receivers with the
 * receiver residuals as lam).  All arrays on the device, layouts as in
 * vsie_source_sums; out is n x nrhs. */
vsie_status vsie_adjoint_rhs(vsie_problem *p, int32_t f, int64_t nrhs, const double *zR, int64_t ldz,
                             const double *ZR, int64_t ldZ, double *out, int64_t ldo, void *stream);

/* Gradient of a real receiver misfit J with respect to the per-cell sound
 * speed and density of the problem's current materials, for nrhs forward
 * solutions P (A_f P = b) and adjoint solutions lam (A_f^H lam = E^H rho,
 * rho the conjugate-Wirtinger gradient of J with respect to the receiver
 * pressures p_rec = p_inc - E P).  z, Z: vsie_source_sums of lam over the
 * collocation points; zR, ZR: vsie_source_sums of rho over the receivers.
 * Writes grad_c and grad_rho (DEVICE, n_vol doubles each), summed over the
 * right-hand sides:
 *   dJ = Re sum_r [ rho_r^H dE P_r - lam_r^H dA P_r ].
 * The density enters through alpha = rho0/rho - 1 in the single-layer
 * weights, the mass function, the interface jump weights and the grad-alpha
 * neighbour stencil (not differentiated when vgrad_alpha was given; with
 * vgrad_rho, grad alpha = -rho0 grad(rho) / rho^2 varies with the cell's own
 * density while grad(rho) is held fixed). */
vsie_status vsie_param_gradient(vsie_problem *p, int32_t f, int64_t nrhs, const double *P, int64_t ldp,
                                const double *lam, int64_t ldl, const double *z, int64_t ldz,
                                const double *Z, int64_t ldZ, const double *zR, int64_t ldzr,
                                const double *ZR, int64_t ldZr, double *grad_c, double *grad_rho,
                                void *stream);

/* Assembled FP32 operator (the dense block system of section 2.3.4 written
 * once to memory).  Fills `dense`, caller-owned DEVICE memory of 2 * ld * n
 * floats (8 * ld * n bytes), with the off-diagonal entries A_ij of frequency
 * f, computed with the FP64 pair terms and rounded to FP32 (diagonal entries
 * 0), in two column-major planes with leading dimension ld >= n: the real
 * parts at dense[i + j ld], the imaginary parts at dense[ld n + i + j ld].
 * Until vsie_release_dense or vsie_set_materials, every VSIE_FP32 product at
 * frequency f (vsie_matvec, vsie_matvec_adjoint and the inner solves of
 * vsie_solve) multiplies by this matrix on the matrix cores
 * (v_mfma_f32_16x16x4_f32), up to 128 columns per pass: per slab of 8192
 * columns of A (rows for the adjoint) FP32 sums of three real products per
 * complex multiply-add (four with vsie_tuning.mfma_3m = 0), combined and
 * added in FP64 in slab order with the FP64 diagonal.  The memory must stay
 * valid while in use; n and ld must be below 2^31. */
vsie_status vsie_assemble_dense(vsie_problem *p, int32_t f, void *dense, int64_t ld, void *stream);
vsie_status vsie_release_dense(vsie_problem *p, int32_t f);

/* Kernel timing.  vsie_profile(p, 1) clears the counters and starts recording
 * a pair of HIP events around every pair-kernel launch made for p (on the
 * stream of the call that launches it); vsie_profile(p, 0) stops recording.
 * vsie_profile_read synchronises the recorded events and reports, for one
 * kernel kind, the number of launches, their summed duration in ms and the
 * summed pair evaluations (thread points x streamed points per launch; a
 * launch with R right-hand sides counts its pairs once and R in rhs_pairs).
 * kind = 2 * mode + precision with mode 0 forward single layer, 1 forward
 * double layers (T and K), 2 adjoint double layers, 3 adjoint source sums,
 * and precision VSIE_FP64 or VSIE_FP32; kind 8 and 9 are the matrix-core
 * forward single layer and double layers (FP32; a launch over nf frequencies
 * counts nf times its pairs); kind 10 and 11 the symmetric cell-cell single
 * layer in FP64 and FP32 (pairs = ordered cell pairs, n_vol (n_vol - 1));
 * kind 12 and 13 the cell-face kernel in FP64 and FP32 (pairs = 2 n_vol n_srf,
 * both directions); kind 14 and 15 the far-field pattern's single-layer
 * sources, 16 and 17 its double-layer sources, in FP64 and FP32 (pairs =
 * directions x sources); kind 18 and 19 the face-face double layers once per
 * pair in FP64 and FP32 (pairs = n_srf (n_srf - 1)); kind 20 the product with
 * the assembled FP32 operator on the matrix cores (pairs = n^2 entries,
 * rhs_pairs = n^2 nrhs complex multiply-adds per pass of at most 128
 * columns); kind 21 and 22 the FP64 matrix-core forward single layer and
 * double layers (pairs as kinds 8 and 9). */
typedef struct {
    int64_t launches;
    double ms;
    double pairs;
    double rhs_pairs;
} vsie_kernel_stats;
vsie_status vsie_profile(vsie_problem *p, int32_t enable);
vsie_status vsie_profile_read(vsie_problem *p, int32_t kind, vsie_kernel_stats *out);

/* Free the problem and all device memory it owns.  NULL is ignored. */
void vsie_destroy(vsie_problem *p);

/* Message of the calling thread's most recent failed call ("" if none). */
const char *vsie_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* VSIE_H */
