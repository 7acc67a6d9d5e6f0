/*
 * gplmm.h -- C ABI of the MI355X gPLMM Newton-Krylov solver.
 *
 * The library solves the MAC-staggered incompressible Navier-Stokes equations
 * on a voxel image of a porous material (Li & Mehmani, "Preconditioning and
 * Reduced-Order Modeling of Navier-Stokes Equations in Complex Porous
 * Microstructures"):
 *   Section 1, the governing equations and the Newton system
 *     J^k delta^k = -r^k,  J = [F G^T; G O];
 *   Section 2, the MAC discretisation on the image voxels;
 *   Sections 3.1-3.2, the two-level monolithic preconditioner
 *     M^-1 = M_G^-1 + M_dp^-1 (I - A M_G^-1)
 *   with the PLMM coarse operator M_G (reduction, prolongation, restriction,
 *   Remark 1) and the dual-primary Schwarz smoother M_dp;
 *   Section 4, gPLMM: A := J~_w, the Jacobian of the modified residual with
 *   the inertia linearised about a wind w and removed on faces near the
 *   contact interfaces;
 *   Section 8, right-preconditioned (flexible) GMRES with the tolerance
 *   measured against ||r(u = 0, p = 0)||.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Image arrays are indexed [k][j][i] (z, y, x) with x fastest, nx*ny*nz bytes
 * or int32 words; nz = 1 means a 2D image.  mask[v] = 1 marks a void (fluid)
 * voxel.  pore_labels[v] > 0 on every void voxel (the watershed pores).
 * Only the largest face-connected void component is kept (periodic axes
 * wrap); every other voxel is treated as grain.
 *
 * Unknown layout ("cell records"): the kept fluid cells are numbered
 * c = 0..ncell-1 in raster order; cell c owns the record
 *   slots [nrec*c, nrec*c + nrec),  nrec = ndim + 1,
 * holding the velocity on the LOWER face of the cell along x, y (, z) and then
 * the pressure.  The lower x-face of cell (k,j,i) lies between cells
 * (k,j,i-1) and (k,j,i).  A face is an unknown only when both its cells are
 * kept fluid; the slot of an inactive face is a "void slot" that must hold 0
 * in every vector passed in, and holds 0 in every vector the library writes.
 * N = nrec * ncell.  gplmm_get_maps() returns the voxel of each cell.
 *
 * Vectors named *_dev are caller-owned device buffers of N doubles on the
 * context's stream, which the library reads or writes in stream order.  The
 * library owns every internal buffer (factors, Krylov basis, coarse operator)
 * and frees them in gplmm_destroy().  Host arrays passed to setup are copied.
 *
 * Errors: every call returns 0 on success, a positive value when a solve ran
 * but missed its tolerance, and a negative GPLMM_E* code on failure; nothing
 * throws across the ABI.  gplmm_last_error() describes the last failure.  One
 * context serves one stream; calls on one context must not overlap.
 */
#ifndef GPLMM_H
#define GPLMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gplmm_ctx gplmm_ctx;

enum {
    GPLMM_OK = 0,
    GPLMM_E_ARG = -1,        /* bad argument (null pointer, size, label) */
    GPLMM_E_GEOMETRY = -2,   /* no fluid, or a decomposition that cannot be built */
    GPLMM_E_HIP = -3,        /* a HIP runtime call failed */
    GPLMM_E_BREAKDOWN = -4,  /* zero or non-finite pivot in a local factorisation */
    GPLMM_E_STATE = -5       /* call order (e.g. apply before build) */
};

enum { GPLMM_FP64 = 0, GPLMM_FP32 = 1 };

/* Wind of the build matrix X = J~_w (Section 4).  The paper uses the velocity
 * at a nearby state and falls back to the Stokes velocity. */
enum {
    GPLMM_WIND_ZERO = 0,     /* w = 0: X is the Stokes (or transient Stokes) matrix, built once */
    GPLMM_WIND_STOKES = 1,   /* w = 0 for the first Newton step, then rebuilt once with the
                                velocity after that step (the Stokes solution) */
    GPLMM_WIND_CALLER = 2    /* w set by gplmm_build(ctx, w_dev) and kept */
};

/* Matrix the preconditioner is built from (the A-hat of Sections 3.1-3.2). */
enum {
    GPLMM_BUILD_GEOMETRIC = 0,  /* gPLMM (Section 4): X = J~_w, the Oseen operator of the wind
                                   with no inertia on tagged faces */
    GPLMM_BUILD_JACOBIAN = 1    /* aPLMM (Sections 3 and 8): the Newton Jacobian J(w) at the build
                                   state w, untagged.  With GPLMM_WIND_ZERO it is the Stokes matrix
                                   (aPLMM_S, which equals gPLMM with w = 0); with GPLMM_WIND_STOKES it
                                   is rebuilt once from J at the first Newton iterate (aPLMM_NS) */
};

typedef struct {
    int nx, ny, nz;          /* image size; nz = 1 for 2D */
    double h;                /* voxel edge (default 1) */
    int periodic[3];         /* per axis x, y, z (default 1, 0, 0) */
    int precision;           /* GPLMM_FP64 (plain) or GPLMM_FP32: local factorisations, shape
                                vectors and the preconditioner's inner stencils in FP32 with FP32
                                accumulation; Newton residual, Arnoldi and coarse solve in FP64 */
    int wind_mode;           /* GPLMM_WIND_* (default GPLMM_WIND_STOKES) */
    int tag_layers;          /* faces within this Chebyshev distance of an interface cell carry
                                no inertia in X (default 1) */
    int dual_dilations;      /* face-neighbour growths of each interface into its dual grid;
                                -1 = default (1 in 2D, 0 in 3D) */
    int restart;             /* FGMRES restart length (default 30, at most 1024) */
    double newton_tol;       /* stop when ||r(x)|| <= newton_tol * ||r(0)|| (default 1e-8) */
    double lin_tol;          /* FGMRES stops when ||J d + r|| <= lin_tol * ||r(0)|| (default 1e-9) */
    int newton_maxit;        /* default 30 */
    int lin_maxit;           /* FGMRES iterations per Newton step (default 600) */
    int tile;                /* local factor tile edge: 0 = default (32) */
    int host_only;           /* 1: build the decomposition and index maps on the host only
                                (no device memory; compute calls return GPLMM_E_STATE) */
    void* stream;            /* hipStream_t, NULL = default stream */
    int line_search;         /* 0 (default): full Newton steps x + delta (Section 1); 1: backtracking
                                on ||r||: the update is lambda * delta with lambda = 1, 1/2, ...
                                >= 1/64, the first lambda with ||r(x + lambda delta)|| <=
                                (1 - 1e-4 lambda) ||r(x)|| (the smallest if none).  Either way a
                                step whose residual is not finite is refused: the solve returns
                                GPLMM_E_BREAKDOWN with x at the last finite iterate */
    int use_graph;           /* 1 (default): the preconditioner application is captured once
                                in a HIP graph and replayed (input and output staged through
                                buffers owned by the context); 0: launched kernel by kernel.
                                Timed runs (gplmm_set_timing) always launch kernel by kernel */
    int build_matrix;        /* GPLMM_BUILD_GEOMETRIC (default) or GPLMM_BUILD_JACOBIAN; the
                                residual updates of Eqs. mono_struct_a and Mdp use the same matrix */
    int split_tiles;         /* primaries whose Schwarz block spans more than this many 32-row tiles
                                are solved by one level of nested dissection (two halves cut by a
                                separator plane, solved in parallel, and the separator's Schur
                                complement); 0 (default) or -1 = never.  Single images only.  It
                                shortens the longest substitution chain but adds the separator
                                rows and a second launch: slower on the 128^3 packing */
    int mg_form;             /* coarse correction: 0 (default) the compact form of Remark 1,
                                Phat (Rhat X Phat)^-1 Rhat with the f unknowns left at zero;
                                1 the full form of Eq. iMG, the coarse operator Rhat Xcheck Phat
                                from the column-summed matrix (the two reductions of Section
                                3.2.2 applied to X) and the f unknowns from the back-substitution
                                of Eq. xf; 2 the compact form followed by the same
                                back-substitution of Eq. xf.  With 1 and 2 every application
                                solves the diagonal blocks of A^f_f and applies X once more.
                                Single images only; not with split_tiles */
} gplmm_options;

typedef struct {
    int ndim, nrec;
    int64_t ncell, N;        /* kept fluid cells; vector length */
    int64_t nface_active;    /* velocity unknowns */
    int Np, Nc, Ny;          /* primaries, contact interfaces, coarse correction unknowns */
    int64_t pin;             /* cell whose mass row is replaced by p = 0 (first sample's in a batch) */
    int64_t ndual_cells;     /* cells covered by at least one dual grid */
    int64_t local_unknowns;  /* sum of the local problem sizes (closure, primary, dual) */
    int64_t factor_bytes;    /* device bytes held by the local factors */
    int ncolors;             /* probing colours used to assemble the coarse operator */
    double lu_flops;         /* flops of the local factorisations of one build: 2 T^3 per tile
                                product of the closure, dual, primary and separator LU schedules */
    int nsplit;              /* primaries solved by nested dissection (options.split_tiles) */
    int64_t sep_unknowns;    /* unknowns on their separators */
    int nfblock;             /* options.mg_form 1, 2: diagonal blocks of A^f_f (connected f-face sets) */
    int max_fblock;          /* unknowns of the largest of them */
    int64_t f_unknowns;      /* f-faces (velocity unknowns owned by no primary) */
} gplmm_layout;

typedef struct {
    int newton_its;
    int lin_its_total;
    int lin_its[64];         /* FGMRES iterations of each Newton step */
    double res_hist[65];     /* ||r(x_k)|| / ||r(0)||, k = 0..newton_its */
    double r0_norm;
    double t_build_ms;       /* preconditioner builds (local factorisations + coarse) */
    double t_solve_ms;       /* FGMRES time */
    double t_total_ms;
    int builds;
    int converged;
    int gs_reorth;           /* Arnoldi steps that needed a second Gram-Schmidt projection */
    double step_length[64];  /* Newton step length lambda of each Newton step */
    double t_coarse_ms;      /* coarse-operator assembly (probing or learned inference), all builds */
    int learned_builds;      /* builds whose coarse operator came from the learned model */
    int coarse_fallbacks;    /* Newton steps redone with the exact coarse operator */
} gplmm_stats;

/* Fill *opt with the defaults listed above. */
void gplmm_default_options(gplmm_options* opt);

/* Build the geometry, the unknown numbering and the pore decomposition
 * (Section 3.2.1: primary grids, contact interfaces, dual grids; Section 4:
 * tagged faces) from a host mask and host pore labels, and upload them.
 * rho, mu: density and viscosity; body[3]: body force per unit mass;
 * dt > 0 selects one backward-Euler step of that size, dt <= 0 the steady
 * equations.  On success *out receives a new context.
 * Errors: GPLMM_E_ARG (null pointers, dims, labels <= 0 on fluid voxels),
 * GPLMM_E_GEOMETRY (no fluid), GPLMM_E_HIP. */
int gplmm_setup(const uint8_t* mask, const int32_t* pore_labels, double rho, double mu,
                const double body[3], double dt, const gplmm_options* opt, gplmm_ctx** out);

/* The pore-network decomposition (Section 3.3, the PNM variant of the preconditioner):
 * the primary grids are throat regions and each contact interface sits in a pore body,
 * shared by every throat that meets there.  throat_labels[v] > 0 on the fluid voxels (the
 * throat regions, e.g. a watershed seeded at the pores' contact pixels); pore_labels[v] > 0
 * on the fluid voxels (the pore decomposition): a cell carved by the rule of gplmm_setup
 * applied to throat_labels joins the interface of its pore label (one interface per pore
 * label present among the carved cells, numbered in label order).  Every other step (tags,
 * dual grids, closures, coarse operator, smoothers) is that of gplmm_setup, so any
 * build_matrix or wind option gives the corresponding gPNM / aPNM preconditioner.  Single
 * images only.  Errors as gplmm_setup, and GPLMM_E_ARG for a carved cell without a
 * positive pore label. */
int gplmm_setup_pnm(const uint8_t* mask, const int32_t* throat_labels, const int32_t* pore_labels, double rho,
                    double mu, const double body[3], double dt, const gplmm_options* opt, gplmm_ctx** out);

/* A batch of independent samples in one context (many samples of uneven size solved
 * together: every kernel launch covers all subdomains of all samples).  Sample s is the
 * host image masks[s] / labels[s] of dims[3s..3s+2] = (nx, ny, nz) voxels (nz = 1 for 2D;
 * all samples 2D or all 3D, each axis <= 1024), with its own rho[s], mu[s], body force
 * body[3s..3s+2] and backward-Euler step dt[s] (dt may be NULL: all steady).  The
 * periodicity, h and every other option come from *opt and apply to every sample.  Each
 * sample is decomposed exactly as gplmm_setup decomposes it alone (Section 3.2.1);
 * the batch numbers the cells, primaries and interfaces of sample s after those of
 * samples 0..s-1 (offsets from gplmm_batch_info), and voxels in the concatenation of
 * the images.  Each sample keeps its own pinned cell.  The batch is one block-diagonal
 * system: the coarse operator has one dense block per sample.  gplmm_newton_solve runs one
 * FGMRES Arnoldi process per sample in lockstep (the preconditioner and Jacobian launches
 * cover all samples; dot products, Hessenberg matrices and stopping tests are per sample)
 * to lin_tol ||r_s(0)|| on every sample s, and stops Newton at newton_tol ||r_s(0)||;
 * res_hist holds max_s ||r_s(x_k)|| / ||r_s(0)||, lin_its the lockstep iterations (those
 * of the slowest sample), and the line search backtracks per sample.
 * 1 <= nsamples <= 1024.  Errors as gplmm_setup; the message names the sample. */
int gplmm_setup_batch(int nsamples, const uint8_t* const* masks, const int32_t* const* pore_labels,
                      const int32_t* dims, const double* rho, const double* mu, const double* body,
                      const double* dt, const gplmm_options* opt, gplmm_ctx** out);

/* Offsets of the samples of a batch (a single-image context is a batch of one): arrays
 * of nsamples + 1 entries, owned by the caller, any may be NULL: cell_off (kept cells;
 * the vector slots of sample s are [nrec cell_off[s], nrec cell_off[s+1])), voxel_off
 * (concatenated images), prim_off, iface_off. */
int gplmm_batch_info(const gplmm_ctx* ctx, int* nsamples, int64_t* cell_off, int64_t* voxel_off,
                     int32_t* prim_off, int32_t* iface_off);

/* out_host[s] = ||r_s(x)|| / ||r_s(0)|| for every sample s (one entry for a single image):
 * the relative residual each sample reached. */
int gplmm_sample_residuals(gplmm_ctx* ctx, const double* x_dev, const double* x_prev_dev, double* out_host);

/* Sizes of the layout and of the decomposition. */
int gplmm_layout_info(const gplmm_ctx* ctx, gplmm_layout* out);

/* Host copies of the index maps (arrays sized by gplmm_layout_info):
 * cell_voxel[ncell]   voxel (raster index) of each kept fluid cell;
 * cell_iface[ncell]   contact interface of each cell, -1 for primary cells;
 * cell_prim[ncell]    primary grid of each cell, -1 for interface cells;
 * face_owner[N]       for velocity slots: owning primary, -1 for f-faces (both cells
 *                     in interfaces), -2 for void slots; for pressure slots: -3;
 * face_tag[N]         bit 0: the velocity slot carries no inertia in X (tagged face);
 *                     bit 1: the face belongs to a wall-free group of its primary and keeps
 *                     its plain row in the closure matrix.
 * Any pointer may be NULL to skip that map. */
int gplmm_get_maps(const gplmm_ctx* ctx, int32_t* cell_voxel, int32_t* cell_iface,
                   int32_t* cell_prim, int32_t* face_owner, int8_t* face_tag);

/* Dual grid membership: dual_ptr[Nc+1], dual_cells[dual_ptr[Nc]] (cells of each dual
 * grid, ascending).  Call with dual_cells = NULL to get dual_ptr only. */
int gplmm_get_duals(const gplmm_ctx* ctx, int64_t* dual_ptr, int32_t* dual_cells);

/* Sizes of the local problems of Section 3.2.3 (primaries first, in primary order, then
 * the dual grids in interface order; Np + Nc entries each): n[s] local unknowns and
 * factor_elems[s] stored factor elements (diagonal tiles, L tile rows, U tile columns).
 * Host arrays owned by the caller; either may be NULL. */
int gplmm_get_subdomains(const gplmm_ctx* ctx, int32_t* n, int64_t* factor_elems);

/* Nested-dissection plan of split k, 0 <= k < layout.nsplit (options.split_tiles): info[4]
 * = {primary, nA, nB, nS}, and, when slots is not NULL (nA + nB + nS entries), the record
 * slots of the primary's unknowns in their elimination order: half A, half B (in its own
 * order, the cut plane last), then the separator S.  A and B are uncoupled in X, nA and nB
 * are multiples of the tile, and every pressure follows its faces, so the block
 * factorises without pivoting in this order as two independent halves and the
 * separator's Schur complement.  Host arrays owned by the caller; GPLMM_E_ARG for k out
 * of range. */
int gplmm_get_split(const gplmm_ctx* ctx, int k, int32_t* info, int32_t* slots);

/* Diagonal blocks of A^f_f used by the back-substitution of Eq. xf (options.mg_form 1, 2):
 * the f-faces (velocity unknowns owned by no primary) grouped into the connected sets of
 * X's couplings among them, so that A^f_f is block diagonal over the blocks.  ptr
 * (layout.nfblock + 1 entries) gets the offsets of the blocks in slots; slots
 * (layout.f_unknowns entries, may be NULL) the record slots of each block, ascending.
 * Host arrays owned by the caller; with mg_form 0 there are no blocks (ptr[0] = 0). */
int gplmm_get_fblocks(const gplmm_ctx* ctx, int64_t* ptr, int32_t* slots);

/* r = r(x): the MAC residual of the momentum and mass equations (Section 1;
 * backward Euler against x_prev when dt > 0, x_prev may be NULL = 0; the pinned
 * cell's mass row is p = 0).  All pointers are device vectors of N doubles. */
int gplmm_residual(gplmm_ctx* ctx, const double* x_dev, const double* x_prev_dev, double* r_dev);

/* y = J(xlin) v: the Newton Jacobian of gplmm_residual at xlin, upwind
 * branches frozen at xlin (Section 1, the Newton system). */
int gplmm_matvec(gplmm_ctx* ctx, const double* xlin_dev, const double* v_dev, double* y_dev);

/* y = X v with the current build matrix X = J~_w (Section 4). */
int gplmm_build_matvec(gplmm_ctx* ctx, const double* v_dev, double* y_dev);

/* Build the gPLMM preconditioner from X = J~_w with wind w (device vector, NULL
 * = zero wind): assemble and factorise every local problem (closure matrices of
 * the primaries, primary and dual Schwarz blocks), form shape and correction
 * vectors (Section 3.2.2, prolongation), assemble and invert the coarse operator
 * Rhat X Phat (Remark 1).  Errors: GPLMM_E_BREAKDOWN, GPLMM_E_HIP. */
int gplmm_build(gplmm_ctx* ctx, const double* wind_dev);

/* Host copy of the coarse operator Rhat X Phat assembled by the last gplmm_build
 * (row-major, nco x nco with nco = Nc + Ny; rows and columns: interfaces 0..Nc-1,
 * then the correction unknowns of the primaries that carry one, in primary order).
 * ao_host must hold nco*nco doubles; nco_out (may be NULL) receives nco. */
int gplmm_get_coarse(gplmm_ctx* ctx, double* ao_host, int* nco_out);

/* z = M^-1 v (Section 3.1 with Section 3.2.3: coarse correction, then the dual
 * and the primary additive-Schwarz smoothers).  Requires gplmm_build.  v_dev and
 * z_dev must not alias. */
int gplmm_precond_apply(gplmm_ctx* ctx, const double* v_dev, double* z_dev);

/* Newton-FGMRES with gPLMM.  x_dev: in = initial guess, out = solution.
 * x_prev_dev: previous time level for dt > 0 (NULL = 0).  Builds the
 * preconditioner as wind_mode asks.  stats may be NULL.  Returns 0 when
 * ||r|| <= newton_tol ||r(0)||, 1 when the iteration limit was reached. */
int gplmm_newton_solve(gplmm_ctx* ctx, const double* x_prev_dev, double* x_dev, gplmm_stats* stats);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the norms of gplmm_sample_residuals,
 * out_dev[s] = ||r_s(x)|| / ||r_s(0)|| (||r_s(x)|| when r_s(0) = 0), written to a
 * caller-owned device array of nsamples doubles in stream order, with no allocation, no
 * host copy and no synchronisation.  x_dev, x_prev_dev (NULL = 0): device vectors of N
 * doubles.  The partial sums live in a static 1 MiB device array that every call on the
 * same GPU shares (at most 65536 samples; a batch holds at most 1024): calls that overlap
 * on one GPU race.  Errors: GPLMM_E_ARG, GPLMM_E_STATE (host-only context), GPLMM_E_HIP. */
int gplmm_sample_residuals_noalloc(gplmm_ctx* ctx, const double* x_dev, const double* x_prev_dev, double* out_dev);

/* Coarse-scale Navier-Stokes solver (Section 5, Algorithm 1): an approximate steady
 * solution from Newton iterations on the coarse unknowns alone.  The body force is
 * raised in `increments` equal steps to its full value (the paper raises the inlet
 * pressure; the steps play the role of its Reynolds-number increments).  At each step
 * Phat and Rhat are built from X = J~_w with w = the velocity of the previous step
 * (zero at the first: the Stokes matrix), and Newton iterates
 *   J_c delta_c = -r_c,  r_c = Rhat r~(x),  J_c = Rhat J~(x) Phat,  x <- x + Phat delta_c,
 * r~ being the residual without inertia on tagged faces and J~ its Jacobian, until
 * ||r_c|| < tol ||r_c^0|| (the paper's 1e-6).  x_dev (device, N doubles) receives the
 * approximate solution (its input value is ignored: Algorithm 1 starts at rest).
 * Single-image steady contexts with at least one tag layer and one coarse unknown.  The
 * context's preconditioner is left unbuilt (the next solve or gplmm_build rebuilds it).
 * Errors: GPLMM_E_ARG (batch, transient, tag_layers < 1, no coarse unknown, options),
 * GPLMM_E_BREAKDOWN (singular local or coarse factorisation), GPLMM_E_HIP.  Returns 1
 * when a step missed the tolerance within newton_maxit iterations. */
typedef struct {
    int increments;          /* body-force steps (default 1, at most 64) */
    int newton_maxit;        /* coarse Newton iterations per step (default 50) */
    double tol;              /* ||r_c|| < tol ||r_c^0|| ends a step (default 1e-6) */
} gplmm_coarse_options;

typedef struct {
    int increments;
    int newton_its[64];      /* coarse Newton iterations of each step */
    double rc_rel[64];       /* ||r_c|| / ||r_c^0|| reached at each step */
    double fine_rel_residual;/* ||r(x)|| / ||r(0)|| of the returned state (the true residual) */
    double t_build_ms;       /* preconditioner builds (one per step) */
    double t_total_ms;
    int converged;
} gplmm_coarse_stats;

void gplmm_coarse_default_options(gplmm_coarse_options* opt);
int gplmm_coarse_solve(gplmm_ctx* ctx, const gplmm_coarse_options* opt, double* x_dev, gplmm_coarse_stats* stats);

/* Reynolds-number continuation (the protocol of Section 8: the driving force raised in
 * steps, Newton warm-started from the previous step, the preconditioner of each step built
 * from the previous step's velocity).  The body force of step k is scales[k] times the
 * context's; scales increase within (0, 1] and end at 1.  Step 0 runs gplmm_newton_solve
 * from x as given (wind by options.wind_mode); step k > 0 builds once with w = x and runs
 * Newton from x.  x_dev (device, N doubles) is the initial state in and the solution at the
 * full force out; stats (host, steps entries) receives each step's statistics (its build
 * counted in t_build_ms and builds).  Single steady images only.  Returns 0 when every step
 * converged, 1 when a step stopped unconverged (later steps are not run), < 0 on error;
 * the context's body force and wind mode are restored either way. */
int gplmm_continuation(gplmm_ctx* ctx, int steps, const double* scales, double* x_dev, gplmm_stats* stats);

/* Progress report of long solves: fn(user, k, its, rel) is called on the host after every
 * FGMRES restart cycle of Newton step k (its = FGMRES iterations of the step so far,
 * rel = -1) and after every Newton step (its = the step's FGMRES iterations, rel = the
 * relative residual reached, max over the samples of a batch).  fn = NULL stops the
 * reports.  The callback must not call back into the library. */
typedef void (*gplmm_progress_fn)(void* user, int newton_it, int lin_its, double rel);
int gplmm_set_progress(gplmm_ctx* ctx, gplmm_progress_fn fn, void* user);

/* Record HIP events around the preconditioner application, the Jacobian
 * stencil and the Arnoldi step (on = 1) or stop recording (on = 0). */
int gplmm_set_timing(gplmm_ctx* ctx, int on);

/* Average device time (ms) and average algorithmic bytes (flops for "lu") of
 * the timed launches of a named kernel group since the last reset, recorded
 * with HIP events on the context's stream (see gplmm_set_timing); used for
 * roofline reporting.  name: "precond_apply", "trsv" (all local solves),
 * "trsv_p" (primary grids; with split primaries its three phases "trsv_p_fwd",
 * "trsv_sep" and "trsv_p_bwd" also, bytes 0), "trsv_d" (dual grids), "trsv_f" (the blocks
 * of A^f_f of options.mg_form 1 and 2), "jv", "arnoldi" (one
 * Gram-Schmidt step), "lu" (one factorisation schedule), and the build phases
 * "build_closure_dual_lu", "build_shape", "build_primary_lu", "build_coarse".
 * Returns the number of samples. */
int gplmm_kernel_time(gplmm_ctx* ctx, const char* name, double* avg_ms, double* bytes);

/* Reset the kernel timers. */
void gplmm_reset_timers(gplmm_ctx* ctx);

const char* gplmm_last_error(const gplmm_ctx* ctx);

void gplmm_destroy(gplmm_ctx* ctx);

/* Launch parameters of the hot kernels chosen by gplmm_autotune. */
typedef struct {
    int red_blocks;          /* blocks of the Krylov dot-product / update kernels */
    int stencil_block;       /* threads per block of the stencil kernels */
    int trsv_mode;           /* primary-grid solves: 0 subdomain solution kept in LDS, one element
                                of each tile per thread; 1 solution in HBM; 2 (default) in LDS,
                                four groups of 256 threads on interleaved tiles, 16-byte loads */
    int from_cache;          /* 1 when read from the cache file instead of measured */
    double t_reduction_ms;   /* best measured Gram-Schmidt step (half a restart cycle of vectors) */
    double t_stencil_ms;     /* best measured X v + J v */
    double t_trsv_ms;        /* best measured dual + primary triangular solves (0 if not built) */
} gplmm_tuning;

/* Measure the candidate launch parameters on this problem (reduction blocks 256..2048,
 * stencil blocks 128/256/512, triangular-solve variant when the preconditioner is
 * built) and keep the fastest for every later call on ctx.  cache_path (may be NULL): a
 * text file of earlier results, one line per (architecture, N, Np, Nc, precision, split
 * primaries); a
 * matching line is used without measuring, a new result is appended.  Calls that
 * overlap on one context race.  Errors: GPLMM_E_STATE (host-only), GPLMM_E_HIP. */
int gplmm_autotune(gplmm_ctx* ctx, const char* cache_path, gplmm_tuning* out);

/* Set the launch parameters directly (red_blocks 64..2048, stencil_block 128/256/512,
 * trsv_mode 0/1/2; the timing fields are ignored).  Errors: GPLMM_E_ARG. */
int gplmm_set_tuning(gplmm_ctx* ctx, const gplmm_tuning* t);

/* ---------------------------------------------------------------------------
 * Learned coarse coefficients: a small MLP (hidden layers of equal width, GELU
 * in its tanh form, linear output) trained by mean-squared error with Adam.
 * The coarse operator it replaces is Rhat X Phat (Section 3.2.2, Remark 1);
 * the exact operator stays the fallback.  Products run on BF16 matrix cores
 * with FP32 accumulation; master weights are FP32.  All x / y / t pointers
 * are device FP32 arrays, row-major [n x nin], [n x nout]; calls run on the
 * stream given at creation (NULL = default stream).
 * ------------------------------------------------------------------------- */
typedef struct gplmm_mlp gplmm_mlp;

/* nin inputs, nlayers hidden layers of nhidden units, nout outputs; max_batch rows
 * per forward chunk and per gradient batch.  Weights start at zero.  Errors:
 * GPLMM_E_ARG (sizes), GPLMM_E_HIP. */
int gplmm_mlp_create(int nin, int nhidden, int nlayers, int nout, int max_batch, void* stream, gplmm_mlp** out);

/* Parameter count of the packed host layout: for each layer (hidden layers first,
 * then the output layer) W (fan_in x fan_out, row-major) then b (fan_out). */
int64_t gplmm_mlp_num_params(const gplmm_mlp* mlp);

/* Copy all parameters from / to a packed host FP32 array; setting them also resets
 * the optimiser state. */
int gplmm_mlp_set_params(gplmm_mlp* mlp, const float* host);
int gplmm_mlp_get_params(gplmm_mlp* mlp, float* host);

/* y = net(x) for n rows (any n, processed in chunks of max_batch). */
int gplmm_mlp_forward(gplmm_mlp* mlp, const float* x_dev, int n, float* y_dev);

/* Mean-squared loss over n <= max_batch rows and its gradient (kept on the device;
 * also copied, packed, to grad_host when it is not NULL). */
int gplmm_mlp_grad(gplmm_mlp* mlp, const float* x_dev, const float* t_dev, int n, double* loss, float* grad_host);

/* One Adam step (Kingma & Ba) with the last gradient. */
int gplmm_mlp_adam(gplmm_mlp* mlp, double lr, double beta1, double beta2, double eps);

/* Minibatch Adam over the n rows in their given order, `epochs` passes; *loss_out
 * receives the mean batch loss of the last pass. */
int gplmm_mlp_train(gplmm_mlp* mlp, const float* x_dev, const float* t_dev, int n, int epochs, int batch,
                    double lr, double* loss_out);

const char* gplmm_mlp_last_error(const gplmm_mlp* mlp);

/* Use a trained model (kCoarse features in, one value out) for the coarse operator of
 * every following build of ctx, NULL = the exact operator (probing of Rhat X Phat).
 * The model predicts asinh(entry / scale) on the structural pattern of the coarse operator
 * (see gplmm_coarse_entries); an operator that cannot be factorised falls back to the
 * exact one, and gplmm_newton_solve redoes a Newton step with the exact operator when
 * FGMRES misses its tolerance.  The model stays owned by the caller and must outlive
 * its use.  GPLMM_E_ARG for a context with options.mg_form 1 (the model predicts the
 * entries of Rhat X Phat). */
int gplmm_set_coarse_model(gplmm_ctx* ctx, gplmm_mlp* model);

/* The structural entries of the coarse operator (row, col: coarse ids, interfaces first,
 * then the primaries' correction unknowns), their features (16 FP32 values per entry,
 * from the geometry and the current wind) and scales, and, when exact != NULL, their
 * values in the last build, which must have used the exact operator (training labels
 * are asinh(exact / scale)).  Call with every array NULL to get *nent.  Host arrays. */
int gplmm_coarse_entries(gplmm_ctx* ctx, int64_t* nent, int32_t* rows, int32_t* cols, float* feat, float* scale,
                         double* exact);

void gplmm_mlp_destroy(gplmm_mlp* mlp);

#ifdef __cplusplus
}
#endif

#endif /* GPLMM_H */
