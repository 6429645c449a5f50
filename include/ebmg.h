/*
 * ebmg.h — C ABI of an embedded-boundary geometric-multigrid elliptic solver
 * for AMD Instinct MI355X (gfx950).
 *
 * Problem (Helmholtz-equations section of Marskar, arXiv:1809.03745):
 *     alpha a(x) phi + beta div( b(x) grad phi ) = rho        on a Cartesian box,
 * Poisson being alpha = 0, beta = -1, b = relative permittivity (eps0 = 1, so
 * rho means rho/eps0, electrodynamic-equations section). The box is cut by
 * embedded boundaries given as signed-distance functions sampled at grid
 * nodes (spatial-discretisation section): electrodes (Dirichlet), at most one
 * dielectric object (a second material whose b is the object's value,
 * coupled to the gas through the multifluid matching condition with surface
 * charge sigma), and insulating walls (Neumann). Each cut cell carries volume
 * fraction, face apertures and centroids, and a linearised boundary facet.
 * The discrete system is the volume-weighted finite-volume form with
 * centroid-interpolated face fluxes and ray-cast / least-squares boundary
 * stencils (boundary-conditions subsection); it is solved by geometric
 * multigrid V-cycles (multigrid-solver subsection) until
 * ||r|| < rtol * ||r0||, r0 being the residual at phi = 0.
 *
 * Conventions (every entry point):
 *  - Cell arrays are float64, contiguous, x fastest: index i + nx*(j + ny*k).
 *  - Pointers documented as DEVICE are on the context's device (e.g. a torch
 *    tensor's data_ptr()); HOST pointers are ordinary CPU memory.
 *  - The caller owns every array it passes; the library keeps no caller
 *    pointer after a call returns, except the DEVICE arrays of a submitted
 *    solve (ebmg_submit), held until its ticket is collected. The library
 *    owns each problem until ebmg_release().
 *  - All device work of a context is ordered on the context's stream. A
 *    context is not thread-safe: one caller thread per context (the
 *    context's own worker thread, which runs submitted solves, aside).
 *  - Errors are reported only through ebmg_status; the library never aborts.
 *    On EBMG_ERR_ARG / EBMG_ERR_GEOMETRY outputs are untouched. On
 *    EBMG_ERR_NOCONV phi holds the last iterate and info is filled.
 *    ebmg_last_error() gives a message owned by the context, valid until the
 *    next call on that context.
 */
#ifndef EBMG_H
#define EBMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EBMG_ABI_VERSION 2

typedef enum {
  EBMG_OK = 0,
  EBMG_ERR_ARG = 1,       /* invalid argument or unsupported configuration   */
  EBMG_ERR_GEOMETRY = 2,  /* saddle / multi-valued / doubly-cut cell, no stencil */
  EBMG_ERR_OOM = 3,       /* device or host allocation failed, or over budget */
  EBMG_ERR_DEVICE = 4,    /* HIP runtime error, or a solve on a host-only context */
  EBMG_ERR_NOCONV = 5,    /* max_cycles reached before the tolerance          */
  EBMG_ERR_NUMERIC = 6,   /* NaN/Inf in inputs or residual growth             */
  EBMG_ERR_BUSY = 7
} ebmg_status;

typedef struct ebmg_ctx_s* ebmg_ctx;
typedef struct ebmg_problem_s* ebmg_problem;
typedef struct ebmg_batch_s* ebmg_batch;
typedef struct ebmg_family_s* ebmg_family;
typedef struct ebmg_mesh_s* ebmg_mesh;
typedef struct ebmg_amr_s* ebmg_amr;

/* Box: dim in {2,3}; n[d] cells per axis (n[2] ignored in 2D); isotropic
 * cell size h; lower corner lo. */
typedef struct {
  int32_t dim;
  int32_t n[3];
  double h;
  double lo[3];
} ebmg_box;

enum { EBMG_OBJ_ELECTRODE = 0, EBMG_OBJ_DIELECTRIC = 1, EBMG_OBJ_WALL = 2 };

/* Embedded object. sdf: HOST, prod(n[d]+1) doubles sampled at nodes
 * lo + (i,j,k) h, x fastest, > 0 outside the object (copied at setup).
 * value: electrode potential / dielectric permittivity / wall outward normal
 * derivative dphi/dn. */
typedef struct {
  int32_t kind;
  double value;
  const double* sdf;
} ebmg_object;

enum { EBMG_BC_DIRICHLET = 0, EBMG_BC_NEUMANN = 1, EBMG_BC_ROBIN = 2 };

/* Domain faces in the order x-, x+, y-, y+, z-, z+. value = Dirichlet value,
 * Neumann outward normal derivative dphi/dn, or Robin a3 in
 * a1 phi + a2 dphi/dn = a3 (n the outward normal). */
typedef struct {
  int32_t kind[6];
  double value[6];
  double robin_a1[6];
  double robin_a2[6];
} ebmg_domain_bc;

enum { EBMG_FP64 = 0, EBMG_MIXED = 1 };

typedef struct {
  double alpha, beta;       /* equation coefficients (Poisson: 0, -1)            */
  double a_gas, a_diel;     /* Helmholtz diagonal a per phase                    */
  double b_gas;             /* gas-phase b; dielectric b is the object's value   */
  int32_t dirichlet_closure;/* 0 linear two-point (default), 1 quadratic          */
  int32_t robin_closure;    /* 0 linear extrapolation (default), 1 Taylor         */
  int32_t eb_order;         /* Dirichlet EB stencil order: 2 (default) or 1       */
  int32_t precision;        /* EBMG_FP64 or EBMG_MIXED (FP32 cycle, FP64 refinement) */
  int32_t nu1, nu2;         /* pre/post smoothing sweeps (0 -> 2)                */
  int32_t bottom_max_dof;   /* coarsen until at most this many unknowns (0 -> 600) */
  int32_t krylov;           /* 0 auto (BiCGStab if any embedded object, else plain
                               V-cycles), 1 plain V-cycles, 2 V-cycle-preconditioned
                               BiCGStab                                          */
  int32_t smoother;         /* 0 autotuned per level at setup, 1 split red and
                               black half-sweeps, 2 fused red+black tile sweep,
                               3 z-marching fused sweep (3D; tile sweep in 2D),
                               4 fixed rule without timing (3D: z-marching
                               sweep on levels of at least 2^23 cells, quad
                               form when the x extent is a multiple of 4; 2D:
                               fused tile sweep where it applies; one-launch
                               colour phases elsewhere);
                               fused sweeps only on levels of at least 32^3 /
                               256^2 cells                                      */
  int32_t tail;             /* coarse levels: 0 autotuned at setup, 1 always by
                               grid-wide launches, 2 always by the one-workgroup
                               engine from the first level of <= 32768 unknowns
                               (batches, level-synchronous: 0 the coarse-part
                               threshold timed at setup, 1 only the bottom level
                               in each box's workgroup, 2 every level of
                               <= 32768 unknowns; 1 and 2 time nothing, so the
                               choice does not depend on concurrent work)       */
  int32_t batch;            /* batched solves (ebmg_setup_batch; one value for all
                               boxes): 0 or 2 level-synchronous (every phase one
                               launch over all boxes, coarse levels per box in
                               one workgroup), 1 one persistent launch with one
                               workgroup per box                                 */
  int32_t graphs;           /* 0: each Krylov iteration / refinement cycle (and
                               each batched iteration) is captured once as a HIP
                               graph on a private stream and replayed on the
                               context stream; 1: kernels launched directly.
                               Both run the same kernels in the same order      */
  int32_t reserved[3];      /* must be zero                                      */
} ebmg_options;

typedef struct {
  int32_t cycles;           /* V-cycles performed                                 */
  int32_t outer_iters;      /* FP64 outer iterations (refinement or BiCGStab)     */
  int32_t levels;
  int32_t n_hist;
  double r0_norm;           /* ||b||_2 (residual at phi = 0)                      */
  double rel_residual;      /* final ||b - A phi||_2 / ||b||_2 (FP64)             */
  double seconds;           /* wall time of the solve call                        */
  int64_t est_bytes;        /* estimated device-memory bytes the solve's kernels
                               must move (algorithmic: each kernel's minimum
                               reads and writes, summed over its launches);
                               est_bytes / seconds is the solve's effective
                               bandwidth                                         */
  double hist[64];          /* relative residual after each cycle                 */
} ebmg_solve_info;

/* Fill defaults (Poisson, linear closures, order-2 EB stencils, FP64, V(2,2)).
 * Paper: Helmholtz equations, eq. `helmholtz` (Poisson: alpha = 0, beta = -1
 * with eps0 = 1). */
void ebmg_default_options(ebmg_options* opt);

/* EBMG_ABI_VERSION of the built library (no paper passage). */
int ebmg_abi_version(void);

/* Create a context (no paper passage: the device and stream every later call
 * runs on) on a HIP device with a caller stream (NULL = a stream the
 * library creates at default priority). device < 0 gives a host-only context
 * that can set up and export problems but cannot solve (EBMG_ERR_DEVICE). */
ebmg_status ebmg_create(int32_t device, void* hip_stream, ebmg_ctx* out);
/* End the context handle (no paper passage): queued submitted solves run to
 * completion first.
 * Problems and batches set up on the context stay usable until released;
 * the context's stream and worker thread go with the last of them. */
ebmg_status ebmg_destroy(ebmg_ctx ctx);
/* Message of the last failing call on ctx; with ctx == NULL, of the calling
 * thread's last failing ebmg_create (no paper passage; owned by the library). */
const char* ebmg_last_error(ebmg_ctx ctx);

/* Build geometry moments, the finest-level operator (cut-cell rows), the
 * multigrid hierarchy and the bottom-level inverse on the host, and upload
 * them (device contexts). Boundary-condition TYPES and object kinds are fixed
 * here; values may change per solve.
 * Paper: Spatial discretization (cut cells from a level set: volume
 * fractions, apertures, centroids, linearised facets); Helmholtz equations
 * (eq. `poisson_integral` over a cut cell, centroid-interpolated face
 * fluxes, eq. `matching` for the dielectric interface) and its Boundary
 * conditions (domain closures, eq. `bndry_stencil` with the ray casting of
 * figure `raycast` and the least-squares fallback, Robin extrapolation);
 * Multigrid solver (the coarsened hierarchy). box, objs (with their HOST
 * sdf arrays), bc and opt are HOST and are copied; *out receives the
 * problem. ERR_ARG for an invalid box or option, ERR_GEOMETRY for cells the
 * discretisation cannot represent (saddles, cells cut by two objects, cut
 * cells without a stencil), ERR_OOM / ERR_DEVICE from the upload; on error
 * *out is untouched. */
ebmg_status ebmg_setup(ebmg_ctx ctx, const ebmg_box* box, int32_t nobj, const ebmg_object* objs,
                       const ebmg_domain_bc* bc, const ebmg_options* opt, ebmg_problem* out);

/* Sizes: cells, second-phase unknowns (the dielectric side of interface
 * cells; Paper: Multigrid solver, a patch cut by a multifluid boundary
 * carries both phases), levels, device bytes held. Outputs HOST, any may be
 * NULL. */
ebmg_status ebmg_query(ebmg_problem pb, int64_t* n_cells, int64_t* n_phase2, int32_t* n_levels,
                       int64_t* device_bytes);

/* Sizes of multigrid level `level` (0 = finest; Paper: Multigrid solver):
 * cells and second-phase unknowns. Outputs HOST. ERR_ARG for a bad level. */
ebmg_status ebmg_query_level(ebmg_problem pb, int32_t level, int64_t* n_cells, int64_t* n_phase2);

/* Measurement record of the smoother autotuner (Paper: Multigrid solver, the
 * red/black Gauss-Seidel relaxation). Outputs HOST.
 * Smoother choice of level `level` (0 split half-sweeps, 1 fused tile sweep,
 * 2 + c z-marching fused sweep in tile configuration c as listed at
 * ebmg_smooth, 16 one-launch colour phases), the split sweep time and the
 * chosen (or best
 * fused) variant's sweep time (ms) as the setup autotuner measured them (0 if
 * not timed).
 * level = -1 reports the coarse-tail choice instead: *fused receives the first
 * level run by the one-workgroup engine (-1: none), *split_ms the V-cycle time
 * without it and *fused_ms the V-cycle time with the chosen tail. */
ebmg_status ebmg_query_tuning(ebmg_problem pb, int32_t level, int32_t* fused, double* split_ms, double* fused_ms);

/* Paper: Multigrid solver (the coarsened levels).
 * HOST copies of a level's cell tags (0/1 regular gas/dielectric, 2 explicit
 * row, 3 covered; +4 when the cell's children do not all map to its primary
 * unknown), primary phase per cell and cell of each second-phase unknown
 * (the coarsened graph of the Multigrid solver subsection). Arrays of the
 * level's sizes (ebmg_query_level), caller-owned; any may be NULL. */
ebmg_status ebmg_export_level(ebmg_problem pb, int32_t level, uint8_t* tag, int8_t* primary, int64_t* sec_cell);

/* HOST copies of geometry for cross-checks (Paper: Spatial discretization, volume
 * fractions; the gas-side unknown is the primary one of a two-phase cell).
 * kappa: N per phase (phase 0/1); primary: N int8 (0 gas, 1 dielectric, -1
 * covered); sec_cell: n_phase2 int64 cell of each second-phase unknown. Any
 * pointer may be NULL. */
ebmg_status ebmg_export_geometry(ebmg_problem pb, double* kappa_gas, double* kappa_diel,
                                 int8_t* primary, int64_t* sec_cell);

/* HOST copies of the cut-cell moments of phase `phase` (0 gas, 1 dielectric)
 * for cross-checks. Paper: Spatial discretization (volume fractions, face
 * area fractions and the linearised boundary facet of each cut cell, from
 * the level set sampled at the nodes) and Helmholtz equations (the face
 * centroids that fluxes are interpolated to, the facet centroid and normal
 * where the EB flux is evaluated).
 *  vcent     dim*N, component-major: volume centroid (absolute coordinates);
 *            the cell centre for full cells, 0 where the phase is absent.
 *  apert     face aperture alpha in [0,1] of every face, faces normal to x
 *            first, then y, then z; the faces normal to d form an array of
 *            (n_x + [d=0]) x (n_y + [d=1]) (x (n_z + [d=2]) in 3D) entries,
 *            x fastest. F = the total face count of the box.
 *  foff      (dim-1)*F, per face (dim-1 consecutive values): the face
 *            centroid's offset from the face centre in units of h along the
 *            face's transverse axes in increasing order; 0 on full or closed
 *            faces.
 *  eb_area   N: facet area / h^(dim-1) (0 without a facet).
 *  eb_cent   dim*N, component-major: facet centroid (absolute coordinates).
 *  eb_normal dim*N, component-major: unit facet normal pointing out of the
 *            phase (0 without a facet).
 * Any pointer may be NULL. ERR_ARG for a phase the problem does not have. */
ebmg_status ebmg_export_moments(ebmg_problem pb, int32_t phase, double* vcent, double* apert, double* foff,
                                double* eb_area, double* eb_cent, double* eb_normal);

/* Paper: Helmholtz equations, Multigrid solver.
 * HOST CSR of the level-`level` operator over N+N2 unknowns (covered cells
 * as identity rows): the linear part of the volume-weighted row of eq.
 * `poisson_integral` (Helmholtz equations) on level 0, the coarse operators
 * of the Multigrid solver subsection elsewhere. Call with row_ptr == NULL to
 * get *nnz only; then row_ptr (N+N2+1), cols and vals (*nnz) are HOST arrays
 * the caller allocates. ERR_ARG for a bad level. */
ebmg_status ebmg_export_operator(ebmg_problem pb, int32_t level, int64_t* nnz, int64_t* row_ptr,
                                 int64_t* cols, double* vals);

/* Paper: Helmholtz equations and its Boundary conditions.
 * HOST right-hand side b (N+N2) for the given data, from the stored boundary
 * coefficients: b = kappa*rho - L(0), i.e. the source of eq.
 * `poisson_integral` plus every boundary datum (domain values, electrode
 * potentials, the surface charge sigma of eq. `matching`). rho: N (primary
 * unknowns); sigma: N or NULL; bc_values: 6 or NULL (setup values);
 * obj_values: nobj or NULL. All HOST. */
ebmg_status ebmg_export_rhs(ebmg_problem pb, const double* rho, const double* sigma,
                            const double* bc_values, const double* obj_values, double* b);

/* Solve. Paper: Multigrid solver (V-cycles with red/black Gauss-Seidel
 * relaxation, stop when ||r|| < lambda ||r0|| with r0 the residual at
 * phi = 0) for the system of Helmholtz equations; E = -grad(phi) from the
 * centroid-interpolated face fluxes (Electrodynamic equations, eq.
 * `poisson`). rho, sigma (nullable), phi (in: initial guess, out: primary
 * unknown per cell; covered cells 0), phi2 (nullable; second-phase
 * unknowns, in/out), E (nullable; dim*N cell-centred field,
 * component-major) are DEVICE arrays. bc_values (6) and obj_values (nobj)
 * are HOST arrays or NULL (setup values). rtol: stop when
 * ||b - A phi||_2 <= rtol ||b||_2. info (HOST, nullable) receives the
 * record. ERR_NOCONV leaves the last iterate in phi; ERR_NUMERIC flags
 * NaN/Inf or residual growth. */
ebmg_status ebmg_solve(ebmg_problem pb, const double* rho, const double* sigma,
                       const double* bc_values, const double* obj_values, double rtol,
                       int32_t max_cycles, double* phi, double* phi2, double* E,
                       ebmg_solve_info* info);

/* Asynchronous solve for serving (no paper passage: the request loop of a
 * solver service; the solve itself is ebmg_solve's): the same solve as
 * ebmg_solve, queued on
 * the context's worker thread (started by the first submit), which runs the
 * submitted solves of a context one after another, in submission order, on
 * the context's stream. Solves on separate contexts (separate streams) run
 * concurrently on the device. Arguments as for ebmg_solve; bc_values and
 * obj_values are copied before the call returns, while rho, sigma, phi,
 * phi2 and E (DEVICE) are used when the solve runs and must stay valid and
 * unwritten by the caller until the ticket has been collected. *ticket
 * (HOST) receives a nonzero id, unique within the context. Argument errors
 * are returned here; errors of the solve itself through poll/wait. Every
 * other call on the problem (ebmg_solve, ebmg_apply, ebmg_set_coefficients,
 * ebmg_release, ...) first waits for its submitted solves to finish.
 * ebmg_destroy runs the queued solves to completion before it returns. */
ebmg_status ebmg_submit(ebmg_problem pb, const double* rho, const double* sigma,
                        const double* bc_values, const double* obj_values, double rtol,
                        int32_t max_cycles, double* phi, double* phi2, double* E,
                        uint64_t* ticket);

/* Non-blocking check of a submitted solve (serving; no paper passage). *done (HOST) = 0 while it is
 * queued or running; once it has finished, *done = 1, *result receives the
 * solve's status (what ebmg_solve would have returned; on failure
 * ebmg_last_error(ctx) gives its message), info (nullable) its record, and
 * the ticket is forgotten. Returns EBMG_ERR_ARG for an unknown or already
 * collected ticket, else EBMG_OK. */
ebmg_status ebmg_poll(ebmg_ctx ctx, uint64_t ticket, int32_t* done, ebmg_status* result,
                      ebmg_solve_info* info);

/* As ebmg_poll, blocking until the submitted solve has finished (serving;
 * no paper passage). */
ebmg_status ebmg_wait(ebmg_ctx ctx, uint64_t ticket, ebmg_status* result, ebmg_solve_info* info);

/* Paper: Helmholtz equations, eq. `poisson_integral`.
 * out = A [phi; phi2]: the linear part of the finest-level operator of the
 * Helmholtz equations section (eq. `poisson_integral`, boundary data
 * excluded), in FP64. phi, phi2, out, out2 are DEVICE arrays of N and N2
 * entries (phi2/out2 nullable when N2 = 0). */
ebmg_status ebmg_apply(ebmg_problem pb, const double* phi, const double* phi2, double* out,
                       double* out2);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * out = A [phi; phi2] as ebmg_apply, computed by the same kernels, with its
 * staging in a fixed device scratch array that the library holds on each GPU
 * from context creation until the process ends (18 MiB), instead of the
 * problem's work vectors. It allocates nothing (no hipMalloc, hipFree or
 * allocating library call) and does not synchronise: the work is queued on
 * the context's stream and out / out2 are ready when that stream reaches it.
 * Limit: N + N2 <= 1179648 unknowns (ERR_ARG beyond). All calls on one GPU
 * share that GPU's scratch, which keeps the last call's contents: calls that
 * overlap on one GPU (several contexts or threads at once) race; serialise
 * them. phi, phi2, out, out2: DEVICE arrays as for ebmg_apply. */
ebmg_status ebmg_apply_noalloc(ebmg_problem pb, const double* phi, const double* phi2, double* out,
                               double* out2);

/* Paper: Electrodynamic equations (eq. `poisson`), Helmholtz equations.
 * Cell-centred E = -grad(phi) (Electrodynamic equations) from the
 * centroid-interpolated face fluxes of the Helmholtz equations section: the
 * mean of the open low/high face gradients per axis, the EB normal gradient
 * where neither face is open. phi, phi2, sigma and E (dim*N,
 * component-major) are DEVICE arrays; bc_values / obj_values HOST or NULL,
 * as in ebmg_solve. */
ebmg_status ebmg_efield(ebmg_problem pb, const double* phi, const double* phi2, const double* sigma,
                        const double* bc_values, const double* obj_values, double* E);

/* Paper: Multigrid solver (red/black Gauss-Seidel relaxation).
 * Red/black Gauss-Seidel sweeps over the template cells of level `level` only: explicit-row,
 * covered and second-phase entries of x are left as they are. variant: 1
 * split red and black half-sweeps, 2 fused tile sweep, 3 + c z-marching
 * fused sweep in tile configuration c = 0..13 (x-by-y tiles over z planes:
 * 64x8 over 32, 64x16 over 32, 32x16 over 32, 64x8 over 16, 128x8 over 32,
 * 32x8 over 32, 32x32 over 32; 7..9: 64x16, 128x8 and 32x32 over 32 with
 * 16-byte fetches, x extent a multiple of 4; 10: 64x16 over 8; 11..13: the
 * quad form, each thread four cells of a row, 64x16, 128x16 and 128x8
 * over 32, x extent a multiple of 4; 3D), 17 one-launch colour
 * phases out of place (four cells of a row per thread when the x extent is
 * a multiple of 4 and the arrays are aligned to four values, else two or
 * one). Every variant performs exactly the red half-sweep
 * followed by
 * the black one with the same arithmetic, so their results agree bitwise.
 * Variant 18 is the one-launch colour phases with the explicit rows
 * included, as the solver smooths levels that use them: in the phase of
 * colour c every template cell of colour c and every explicit row whose
 * cell has colour c (by the parity of i+j+k) is relaxed from the values
 * before the phase. Variant 19 is the level's fused sweep (its chosen
 * configuration, else the z-marching or tile default) followed in every
 * sweep by Jacobi passes over the explicit rows of colour group 0 and then
 * group 1 (group 1 seeing group 0's new values), as the solver smooths
 * levels that use a fused sweep.
 * x (in/out) and b are DEVICE FP64 arrays of the level's N + N2 unknowns;
 * mixed-precision problems sweep in FP32 (x and b rounded, x widened back).
 * Uses the level's work vectors. ERR_ARG where the level cannot use the
 * variant. */
ebmg_status ebmg_smooth(ebmg_problem pb, int32_t level, int32_t variant, int32_t sweeps, double* x,
                        const double* b);

/* Paper: Multigrid solver (restriction of the residual to the coarser
 * level). The V-cycle's residual r = b - A x of level `level` restricted
 * into the right-hand side of level `level` + 1, as a V-cycle forms it
 * (simple coarse cells: the mean of their 2^D children's residuals;
 * non-simple coarse unknowns: their child lists; covered coarse cells: 0).
 * form 0: the solver's own kernels; 1: the fused z-marching kernel in its
 * pair form; 2: separate residual and restriction kernels; all forms agree
 * bitwise (ERR_ARG where a form does not apply to the level). x, b: DEVICE
 * FP64 arrays of the level's N + N2 unknowns; bc: DEVICE FP64 array of the
 * coarse level's N + N2 entries (output). Mixed-precision problems compute
 * in FP32 (x and b rounded, bc widened). Uses the levels' work vectors. */
ebmg_status ebmg_restrict_residual(ebmg_problem pb, int32_t level, int32_t form, const double* x, const double* b,
                                   double* bc);

/* Measurement hook (no paper passage; the kernels are the relaxation and
 * residual of the Multigrid solver subsection): launch one kernel `reps`
 * times on the context stream
 * between two HIP events and report the mean duration per launch (ms) and
 * the kernel's algorithmic bytes per launch. which = 0: the level's chosen
 * smoother kernel; 2: a red/black half-sweep; 3: the level's fused
 * red+black sweep; 4: the z-marching fused sweep (3D); ERR_ARG where the
 * level cannot use a fused sweep -- FP32 for mixed-precision
 * problems, else FP64; 1: FP64 residual of level `level`; 5: a reference
 * stream over the level's arrays with the fused sweep's bytes per cell and
 * no stencil (reads x, b and the tag of every cell, writes one value per
 * cell; ERR_ARG unless N is a multiple of 4). Smoother bytes are
 * 3 values + 1 tag byte per updated cell, residual bytes 3 FP64 values + 1
 * tag byte per cell. Overwrites the level's work vectors. */
ebmg_status ebmg_time_kernel(ebmg_problem pb, int32_t which, int32_t level, int32_t reps, double* avg_ms,
                             double* alg_bytes);

/* Measurement hook, in-solve form (no paper passage): enable = 1 starts
 * timing, inside later
 * ebmg_solve calls on pb, the launches of level `level`'s smoothing-sweep
 * kernel (which = 0: the fused sweep, or each colour phase / half-sweep where
 * the level uses those; not the first z-marching sweep of a V-cycle, which
 * starts from x = 0 and does not read it) or of its FP64 residual kernel (which = 1: the
 * template-cell kernel of the solve's FP64 r = b - A x checks on that level;
 * a V-cycle forms its residual inside the restriction on large 3D levels,
 * elsewhere with the same kernel, then timed as well): each such
 * launch carries a HIP event pair that its dispatch stamps with the
 * kernel's own start and end (extended launch); while any timing is on,
 * those solves launch their kernels directly instead of replaying graphs (the same
 * kernels in the same order). enable = 0 stops it and reports the number of
 * launches timed, their mean duration (ms) and the algorithmic bytes of one
 * launch (as ebmg_time_kernel counts them). Outputs are HOST pointers and may
 * be NULL. ERR_ARG if enable = 0 finds no such timing running on that level. */
ebmg_status ebmg_kernel_timing(ebmg_problem pb, int32_t which, int32_t level, int32_t enable,
                               int64_t* launches, double* mean_ms, double* alg_bytes);

/* Paper: Radiative transfer (eq. `sp1` and its Robin outflow condition,
 * eq. `robin`), Helmholtz equations (its backward-Euler example).
 * Replace the coefficients of a problem without embedded objects and without
 * explicit rows on any level (e.g. the Eddington Helmholtz problem of the
 * radiative-transfer section, kappa phi - div((1/3kappa) grad phi) = S, for a
 * new absorption kappa): alpha, beta, a_gas, a_diel, b_gas in opt and the
 * boundary data in bc (values and Robin a1/a2; kinds must equal those given
 * at setup). Every other option must equal the setup's. The template
 * constants of all levels and the bottom inverse are rebuilt on the host and
 * re-sent; the device hierarchy is kept. ERR_ARG if the problem does not
 * qualify. Not to be called while a solve on the problem is running. */
ebmg_status ebmg_set_coefficients(ebmg_problem pb, const ebmg_options* opt, const ebmg_domain_bc* bc);

/* Free the problem's device hierarchy and host data (waits for its submitted
 * solves first; no paper passage). NULL is ignored. */
ebmg_status ebmg_release(ebmg_problem pb);

/* Batched boxes (independent problems of one dimension and one precision),
 * e.g. the leaves of a patch-based hierarchy (Paper: Spatial discretization,
 * patch-based AMR with fixed-size boxes; each box is discretised as in
 * ebmg_setup). Setup builds every box on the host (in parallel) and uploads
 * it; boxes[i] with nobj[i] objects objs[i], bcs[i] and opts[i] (opts may be
 * NULL for defaults). All arguments HOST, copied. Errors as ebmg_setup,
 * for the first failing box. */
ebmg_status ebmg_setup_batch(ebmg_ctx ctx, int32_t nbox, const ebmg_box* boxes, const int32_t* nobj,
                             const ebmg_object* const* objs, const ebmg_domain_bc* bcs, const ebmg_options* opts,
                             ebmg_batch* out);

/* Total cells, second-phase unknowns and device bytes of a batch (HOST
 * outputs, any may be NULL; no paper passage). */
ebmg_status ebmg_query_batch(ebmg_batch bt, int64_t* cells, int64_t* cells2, int64_t* device_bytes);

/* Cells and second-phase unknowns of box `box` of a batch (HOST outputs,
 * any may be NULL; no paper passage): the sizes of its rho / phi and phi2
 * arrays in ebmg_solve_batch. ERR_ARG for a box index out of range. */
ebmg_status ebmg_query_batch_box(ebmg_batch bt, int32_t box, int64_t* n_cells, int64_t* n_phase2);

/* Measurement record (no paper passage). Setup choices of a batch: mode
 * (1 persistent, 2 level-synchronous), the
 * coarse-part threshold (a box's levels of at most this many unknowns run in
 * one workgroup; 0: only the bottom level), the number of levels run by
 * grid-wide launches, and the timed candidates (up to 8 thresholds and V-cycle
 * ms; ncand receives their count). Any output may be NULL. */
ebmg_status ebmg_query_batch_tuning(ebmg_batch bt, int32_t* mode, int32_t* tail_cells, int32_t* wide_levels,
                                    int32_t* ncand, int32_t* cand_cells, double* cand_ms);

/* Paper: Multigrid solver (as ebmg_solve, per box).
 * Solve every box to ||r|| <= rtol ||b||: right-hand side, FP64 residual,
 * V-cycle (FP32 for mixed precision) as the BiCGStab preconditioner or as
 * plain refinement. With options.batch == 1, in ONE persistent launch:
 * workgroups of 512 threads take boxes (largest first, fixed assignment)
 * and run the whole solve in-group. Otherwise level-synchronous: each phase
 * is one launch over the chunks of all boxes (levels down to a size tuned at
 * setup), each box's coarser levels and bottom solve run in one workgroup,
 * and the Krylov scalars, tests and restarts are kept per box on the device;
 * cycles are then counted in pairs (two preconditioner applications per
 * iteration, also for plain refinement).
 * rho[i], sigma[i] (sigma or its entries may be NULL), phi[i] (in: guess,
 * out: solution) and phi2[i] (may be NULL when the box has no second-phase
 * unknowns) are DEVICE arrays of box i; the pointer arrays themselves are
 * HOST arrays. Boundary values are those given at setup. infos (HOST, nbox
 * entries, may be NULL) receives per-box results; the status is the first
 * non-OK box status. A box's result does not depend on the other boxes. */
ebmg_status ebmg_solve_batch(ebmg_batch bt, const double* const* rho, const double* const* sigma, double rtol,
                             int32_t max_cycles, double* const* phi, double* const* phi2, ebmg_solve_info* infos);

/* Free a batch and every box in it (no paper passage). NULL is ignored. */
ebmg_status ebmg_release_batch(ebmg_batch bt);

/* A family of Helmholtz operators on one geometry, set up once and kept
 * resident: nmem members alpha_k a_k phi + beta_k div(b_k grad phi) = rho_k,
 * each with its own coefficients and domain boundary data.
 * Paper: Radiative transfer (eq. `sp1` solved per frequency group gamma with
 * its own kappa_gamma, outflow condition eq. `robin`) and the Photoionization
 * appendix (three groups with the same source); Parabolic equations (the
 * TGA scheme eq. `tga`: two Helmholtz solves per diffusion step, one per
 * shifted operator I - mu_i L) and the backward-Euler example of the
 * Helmholtz equations section. Every member is discretised as ebmg_setup
 * does (same geometry, objects and boundary kinds); the cut-cell moments are
 * computed once, and members whose operator structure (cell tags, explicit
 * rows and their columns, transfer lists, level by level) equals member 0's
 * use member 0's device copies of that structure, so the family holds one
 * hierarchy structure plus per-member values and vectors. Smoother and
 * coarse-tail choices are member 0's.
 * box, objs (with their HOST sdf arrays): the geometry, as for ebmg_setup.
 * bcs[k], opts[k] (HOST, nmem entries each): member k's domain data and
 * options; the boundary kinds and every option other than alpha, beta,
 * a_gas, a_diel and b_gas must equal member 0's (ERR_ARG otherwise).
 * Errors as ebmg_setup; *out untouched on error. */
ebmg_status ebmg_setup_family(ebmg_ctx ctx, const ebmg_box* box, int32_t nobj, const ebmg_object* objs,
                              int32_t nmem, const ebmg_domain_bc* bcs, const ebmg_options* opts,
                              ebmg_family* out);

/* Sizes of a family (HOST outputs, any may be NULL; no paper passage):
 * members, cells and second-phase unknowns per member, device bytes held by
 * the whole family, and the bytes of structure members take from member 0
 * instead of holding their own copies. */
ebmg_status ebmg_query_family(ebmg_family fam, int32_t* nmem, int64_t* n_cells, int64_t* n_phase2,
                              int64_t* device_bytes, int64_t* shared_bytes);

/* Paper: Multigrid solver (as ebmg_solve, per member). Solve the members
 * whose rho[k] is non-NULL, each to ||r|| <= rtol ||b||, with the setup's
 * boundary values. rho, phi (HOST arrays of nmem pointers) hold DEVICE
 * arrays of N cells (phi in: guess, out: solution); sigma and phi2 may be
 * NULL or hold NULL entries (phi2[k] is required for a member with N2 > 0
 * only when phi2 itself is given). Members run on streams of their own,
 * after the work queued on the context's stream, each driven by its own host
 * thread (the first call runs them one after another); the call returns
 * when all have finished. A member's result does not depend on which other
 * members are solved with it. infos and statuses (HOST, nmem entries, may
 * be NULL) receive each member's record and status; the return value is the
 * first failing member's status (its message in ebmg_last_error). */
ebmg_status ebmg_solve_family(ebmg_family fam, const double* const* rho, const double* const* sigma, double rtol,
                              int32_t max_cycles, double* const* phi, double* const* phi2, ebmg_solve_info* infos,
                              ebmg_status* statuses);

/* Free a family and its members (no paper passage). NULL is ignored. */
ebmg_status ebmg_release_family(ebmg_family fam);

/* Paper: Convection-Diffusion-Reaction equations (Advective discretization,
 * Hybrid divergence). One explicit step n_out = n_in - dt D of the
 * advection of a density on the gas phase of the problem's geometry: D is
 * the divergence of face fluxes u n_f, n_f the upwind state of an unsplit
 * Godunov predictor with van Leer (monotonised-central) slopes extrapolated
 * to the face and the half step (transverse terms included; 0 slope where a
 * neighbour carries no gas); fluxes are interpolated to the face centroids
 * and weighted by the apertures; no flux crosses the embedded boundary;
 * in cut cells the hybrid kappa D^c + (1 - kappa) D^nc (D^nc the
 * kappa-weighted mean over the 3^D block) replaces D^c, and the mass it
 * does not conserve is redistributed over the other gas cells of the block
 * in proportion to their kappa, so that sum kappa n h^D changes by exactly
 * the domain-boundary fluxes. n_in, n_out: DEVICE arrays of N cells
 * (different; cells without gas get 0); u_x, u_y, u_z (u_z NULL in 2D):
 * DEVICE face-normal velocities at the face centres, the faces normal to d
 * forming an (n_x + [d=0]) x (n_y + [d=1]) (x (n_z + [d=2])) array, x
 * fastest; inflow (HOST, 6 or NULL = 0): the density entering through each
 * domain face (x-, x+, y-, y+, z-, z+) where the velocity points inward.
 * The first call on a problem builds and uploads the step's geometry data.
 * Queued on the context's stream and waited for. */
ebmg_status ebmg_advect(ebmg_problem pb, const double* n_in, const double* u_x, const double* u_y,
                        const double* u_z, double dt, const double* inflow, double* n_out);

/* Measurement hook (no paper passage): mean device time of `reps`
 * back-to-back applications, after one untimed one, of the batch's
 * finest-level kernels over every box as a V-cycle runs them: which 0 the
 * template red and black half-sweeps, 1 the explicit-row Jacobi passes of
 * both colour groups. alg_bytes (HOST, may be NULL): their algorithmic bytes
 * per application (template: three values and a tag byte per cell; rows:
 * per stored entry a column index and a value, per row its unknown index,
 * b, diagonal and result). Level-synchronous batches only (else ERR_ARG);
 * overwrites the batch's cycle vectors. */
ebmg_status ebmg_time_batch_kernel(ebmg_batch bt, int32_t which, int32_t reps, double* avg_ms, double* alg_bytes);

/* Composite solves on nested AMR hierarchies. Paper: Numerical methods
 * (patch-based refinement: levels of rectangular boxes, each box inside a
 * box of the next coarser level) and Helmholtz equations (coarse-fine
 * faces: the coarse divergence refluxed with the fine fluxes through the
 * face, held in flux registers). Refinement ratio 2; box 0 is the domain
 * (level 0); a box of level l >= 1 lies inside one box of level l - 1 (its
 * parent), and boxes of one level do not overlap. The unknowns are those of
 * the cells no finer box covers; the operator is every box's own (the
 * domain's boundary conditions on faces that lie on the domain boundary),
 * with, at a coarse-fine face, fine fluxes taken through a ghost value
 * (quadratic along the normal through two fine cells and the parent's
 * quadratic interpolant; one-sided tangential differences where a side is
 * missing) and the coarse face flux replaced by the mean of the fine fluxes
 * on it (refluxing).
 * Setup: boxes (HOST, nbox) with levels (HOST, nbox): box i has cells of
 * size boxes[0].h / 2^levels[i] and corners on its level's lattice; nobj[i]
 * and objs[i] (HOST) the objects sampled on box i's nodes (as for
 * ebmg_setup); bc the domain's conditions; opts shared by every box (the
 * linear Dirichlet closure; precision picks FP64 or FP32 V-cycles). Boxes
 * of levels >= 1 need even corners and sizes >= 4 and must lie two cells
 * inside their parent's coarse-fine faces (else ERR_ARG), and every cell
 * the coarse-fine stencils use (two fine cells inside each coarse-fine
 * face, two coarse cells outside a box, the tangential stencils) must be a
 * regular gas cell no finer box covers, which also keeps boxes of one level
 * from touching: else ERR_GEOMETRY. A host-only context checks all of this
 * and then returns ERR_DEVICE. */
ebmg_status ebmg_setup_amr(ebmg_ctx ctx, int32_t nbox, const ebmg_box* boxes, const int32_t* levels,
                           const int32_t* nobj, const ebmg_object* const* objs, const ebmg_domain_bc* bc,
                           const ebmg_options* opts, ebmg_amr* out);

/* Sizes of box `box` (no paper passage): its cells, second-phase unknowns,
 * the unknowns its children cover, and the device bytes of the whole
 * hierarchy. Any pointer may be NULL. */
ebmg_status ebmg_query_amr(ebmg_amr a, int32_t box, int64_t* n_cells, int64_t* n_phase2, int64_t* n_covered,
                           int64_t* device_bytes);

/* Paper: Multigrid solver (residual reduction to ||r|| <= rtol ||r0||,
 * r0 at phi = 0) applied to the composite system of the hierarchy.
 * rho[i] (DEVICE, N_i doubles) per box; phi[i] (DEVICE, N_i; in: the
 * guess, out: the solution) and phi2[i] (DEVICE, N2_i; may be NULL where a
 * box has none). Right-preconditioned FP64 BiCGStab; the preconditioner is
 * a V-cycle over the boxes: down from the deepest level, one V-cycle of
 * each box on its residual (homogeneous coarse-fine faces) and its parent's
 * residual updated by that correction; one V-cycle of box 0; up again, the
 * parent's correction prolonged and a second V-cycle per box. On return
 * covered cells hold the mean of their children (deepest first). info (HOST, may be NULL): outer_iters the BiCGStab iterations,
 * cycles two per iteration, rel_residual the composite relative residual,
 * est_bytes 0 (not estimated). NOCONV after max_iters, NUMERIC on a
 * non-finite residual; both leave the last iterate. */
ebmg_status ebmg_solve_amr(ebmg_amr a, const double* const* rho, double rtol, int32_t max_iters, double* const* phi,
                           double* const* phi2, ebmg_solve_info* info);

/* Paper: Helmholtz equations (the composite operator with refluxing).
 * out[i] = (A_comp [phi])_i per box (DEVICE arrays as in ebmg_solve_amr);
 * covered unknowns are identity rows (out = phi there). */
ebmg_status ebmg_apply_amr(ebmg_amr a, const double* const* phi, const double* const* phi2, double* const* out,
                           double* const* out2);

/* Free a hierarchy (no paper passage). NULL is ignored. */
ebmg_status ebmg_release_amr(ebmg_amr a);

/* Signed distance from surface tessellations. Paper: Geometry generation
 * (level sets from a watertight two-manifold tessellation held in a doubly
 * connected edge list: the signed distance to the closest polygon, edge or
 * vertex, found by a nearest-first search through a k-d tree of
 * axis-aligned boxes over the polygons).
 * Create: verts (HOST, 3*nvert doubles) and tris (HOST, 3*ntri vertex
 * indices, counter-clockwise seen from outside; polygons are given as
 * triangle fans) are copied; the library builds the half-edge structure,
 * the angle-weighted pseudonormals of faces, edges and vertices (which fix
 * the sign) and the tree, and keeps them on the context's device.
 * ERR_GEOMETRY for a surface that is not a watertight oriented two-manifold
 * (an edge without exactly one opposite half-edge, a degenerate triangle),
 * ERR_ARG for bad sizes or indices, ERR_DEVICE on a host-only context. */
ebmg_status ebmg_mesh_create(ebmg_ctx ctx, int32_t nvert, const double* verts, int32_t ntri, const int32_t* tris,
                             ebmg_mesh* out);

/* Sizes of a resident mesh (HOST outputs, any may be NULL; no paper
 * passage): triangles, tree nodes, tree depth, device bytes. */
ebmg_status ebmg_mesh_query(ebmg_mesh m, int32_t* ntri, int32_t* nnode, int32_t* depth, int64_t* device_bytes);

/* Paper: Geometry generation. The signed distance (> 0 outside the closed
 * surface, < 0 inside) at the nodes lo + (i,j,k) h, 0 <= i <= n[0], ... of
 * a 3D box, written to sdf (DEVICE, prod(n[d]+1) doubles, x fastest: the
 * node-sampled level set ebmg_setup takes for an object, up to the sign
 * convention of the object kind). visits (HOST, nullable) receives the
 * number of tree boxes and triangles the search examined. Work is queued on
 * the context's stream and waited for. */
ebmg_status ebmg_mesh_sdf(ebmg_mesh m, const ebmg_box* box, double* sdf, int64_t* visits);

/* Free a mesh (no paper passage). */
ebmg_status ebmg_mesh_release(ebmg_mesh m);

#ifdef __cplusplus
}
#endif

#endif /* EBMG_H */
