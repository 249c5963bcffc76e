/*
 * pmutdg.h -- C ABI of the MI355X (gfx950) time stepper for PMUT arrays
 * coupled to a DG spectral-element acoustic model (arXiv 2603.06267).
 *
 * One step advances, on the GPU:
 *   - the matrix-free stiffness action of the continuous GLL spectral
 *     elements inside each of (up to) two axis-aligned bricks, or inside one
 *     brick of trilinear hexahedra (Sec. 3, bilinear form a, eq. Wf_2,
 *     volume sum; maps X_K),
 *   - the symmetric interior-penalty terms across the non-conforming,
 *     mixed-order interface Gamma_I between the bricks (eq. Wf_2, interface
 *     sums; penalty gamma_F; interface quadrature on the finer face, Sec. 5),
 *   - the lumped-mass explicit Newmark (beta = 0, gamma = 1/2) update
 *     (Sec. 3.1, eq. semi_SEM, Algorithm 1),
 *   - each PMUT's reduced modal ODE, driven by the applied voltage and by the
 *     pressure it samples on its face, and the face force it returns
 *     (Sec. 2, eq. pmut_problem; Sec. 3.1, eqs. f_i, g_m, semi_PMUT),
 *   - pressure traces at receiver points.
 * At setup, pmdg_match_faces runs the face matching of Sec. 5, Algorithm 3,
 * on the GPU.
 *
 * Conventions
 *   - Every call returns a pmdg_status (0 = OK, negative = error).  No
 *     exception crosses the ABI.  pmdg_last_error() returns a thread-local,
 *     library-owned string describing the last error on the calling thread.
 *   - Host arrays are plain C arrays owned by the caller; the library copies
 *     what it keeps.  Device memory is owned by the caller: the library asks
 *     for one workspace size and sub-allocates inside the buffer passed to
 *     pmdg_bind; it never allocates device memory itself.
 *   - Streams are hipStream_t passed as void*; NULL means the default stream.
 *   - Units are the caller's, but must be consistent (the Python layer uses
 *     mm, us, MHz).
 *   - Layout of the primary brick: PMUT discs sit on its bottom face
 *     z = x0[2]; the secondary brick (if any) sits on top of it and shares the
 *     primary's top face as Gamma_I (the primary is the "+" / fine side).
 *   - Boundaries other than PMUT discs are rigid (homogeneous Neumann)
 *     unless pmdg_set_absorbing or pmdg_set_pml says otherwise.
 *
 * Shape of the interface
 *   - A problem is described in steps rather than one struct: pmdg_create
 *     (mesh, time step, precision, scenario count), then pmdg_set_pmuts,
 *     pmdg_set_pmut_shape (mode shapes, per PMUT, once its face nodes are
 *     known from pmdg_pmut_face_nodes), pmdg_set_drive, pmdg_set_rx,
 *     pmdg_set_receivers and the boundary calls, then pmdg_bind.  Each call
 *     validates its own arguments, so an error names the input at fault.
 *   - Batching (pmdg_batch_create) takes solvers that are already bound
 *     rather than problem descriptions: the batch reuses each solver's
 *     tables, state and traces in place and results are read through the
 *     solvers, so no second copy of a problem exists.
 *   - Traces are read into host memory (pmdg_read_traces) or device memory
 *     (pmdg_read_traces_device).
 *   - A bound solver runs other drives after pmdg_restart (back to step 0,
 *     everything at rest) and pmdg_set_drive, without the set-up of
 *     pmdg_create and the set_* calls again.
 */
#ifndef PMUTDG_H
#define PMUTDG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int pmdg_status;
#define PMDG_OK 0
#define PMDG_EINVAL (-1)    /* bad argument (size, pointer, geometry) */
#define PMDG_ENOMEM (-2)    /* host allocation failed / workspace too small */
#define PMDG_EHIP (-3)      /* a HIP runtime call failed */
#define PMDG_EUNSTABLE (-4) /* time step or PMUT coupling outside the stable range */
#define PMDG_ESTATE (-5)    /* call not allowed in the solver's current state */

typedef struct pmdg_solver pmdg_solver;

/* One axis-aligned brick of ne[0] x ne[1] x ne[2] equal hexahedra carrying a
 * continuous Q_order space on GLL nodes (Sec. 3, spaces V_a^{r_a}). */
typedef struct {
  double x0[3], x1[3]; /* opposite corners, x1 > x0 componentwise */
  int ne[3];           /* elements per axis, >= 1 */
  int order;           /* polynomial order N, 1..8 */
  double c;            /* sound speed (> 0) */
  double rho;          /* density; kappa = rho c^2 of the primary (Sec. 2) */
} pmdg_brick;

typedef struct {
  int ndom;            /* 1 or 2 */
  pmdg_brick dom[2];   /* dom[0] primary (fine); dom[1] secondary (coarse) */
  double cfl;          /* dt = cfl * min_dom(h_min * min GLL gap / 2 / c) if dt <= 0 */
  double dt;           /* explicit time step if > 0 */
  double penalty_alpha;/* SIPG constant alpha in gamma_F (Sec. 3); > 0 */
  int precision;       /* 32: FP32 field state/operators, FP64 ODE+traces; 64: all FP64 */
  int n_scenarios;     /* S >= 1 drive scenarios sharing mesh and PMUT modal data */
  int trace_capacity;  /* steps a solver may take in total (>= 1): receiver samples kept per
                        * receiver and scenario, and length of the per-step drive table */
} pmdg_problem;

/* Creates a solver: builds GLL / Gauss-Legendre rules, the assembled 1D
 * operators, the interface quadrature-point list (fine-face Gauss points
 * mapped into the coarse elements, Sec. 5) and dt.  Rejects geometry where
 * the secondary's bottom face is not the primary's top face (EINVAL) and a
 * dt beyond the explicit stability bound of the volume operator or of the
 * coupled operator with the interface penalty (EUNSTABLE; see
 * pmdg_lambda_max).  *out receives the handle (NULL on error). */
pmdg_status pmdg_create(const pmdg_problem* pr, pmdg_solver** out);

/* PMUTs on the primary's bottom face (Sec. 2, eq. pmut_problem): Np discs
 * with centres ctr[2*Np] (x, y) and radii radius[Np]; per disc Nm modes with
 * angular frequency omega, damping ratio zeta (acting on the predicted modal
 * velocity) and coupling eta, each [Np*Nm] row-major.  Must precede
 * pmdg_bind.  Face nodes inside a disc belong to that PMUT (discs must not
 * overlap: EINVAL). */
pmdg_status pmdg_set_pmuts(pmdg_solver* h, int Np, const double* ctr, const double* radius, int Nm,
                           const double* omega, const double* zeta, const double* eta);

/* Number of face nodes of PMUT k and, if xyz != NULL, their coordinates
 * (xyz[3*n]); the order is the order expected by pmdg_set_pmut_shape. */
pmdg_status pmdg_pmut_face_nodes(pmdg_solver* h, int k, int* n, double* xyz);

/* Mode-shape samples U_{k,m}.n at PMUT k's face nodes, shape[Nm * n]
 * (mode-major).  With the face quadrature weights this defines the coupling
 * matrix B of eqs. f_i and g_m.  Must precede pmdg_bind. */
pmdg_status pmdg_set_pmut_shape(pmdg_solver* h, int k, const double* shape);

/* Drive phi_{k,0}(t) = amp sin(2 pi freq t - phase) * envelope(t), with
 * T_d = ncyc / freq.  amp, phase: [S*Np]; freq: [S].  envelope 0 = smooth
 * window g of Sec. 6.1 (eq. voltage), 1 = rectangular on [0, T_d],
 * 2 = rectangular, never switched off.  May be called before or after bind
 * (after bind it uploads synchronously). */
pmdg_status pmdg_set_drive(pmdg_solver* h, const double* amp, const double* phase, const double* freq,
                           double ncyc, int envelope);

/* TX -> RX switch (Sec. 2, eq. ode): for t > t_switch the voltage is
 * (1/cap) sum_m eta q.  Default t_switch = +infinity (TX only). */
pmdg_status pmdg_set_rx(pmdg_solver* h, double t_switch, double cap);

/* First-order absorbing condition (the surface term int c pdot v ds of the
 * weak form, Sec. 2 and 3.1; C pdot* in the acoustic solve of Algorithm 1)
 * on the outer faces of brick dom given by the 6-bit mask faces: bit 2a for
 * the face at the low end of axis a, bit 2a+1 for the high end.  The
 * interface faces of two coupled bricks (primary top, secondary bottom)
 * cannot be absorbing.  Before bind (PMDG_ESTATE after); PMDG_EINVAL on a
 * bad domain or mask.  Bricks with absorbing faces keep single-step passes
 * (PMDG_OPT_TIME_BLOCK has no effect on them). */
pmdg_status pmdg_set_absorbing(pmdg_solver* h, int dom, int faces);

/* Perfectly matched layer (Sec. 2, eq. full_problem: the damping
 * alpha p_t + beta p, the auxiliary fields Phi and psi with
 * Phi_t = Z1 Phi + c^2 Z2 grad p + c^2 Z3 grad psi, psi_t = p, and the
 * profile zeta_i of that section with constant (c / ell) log(1 / R)) inside
 * brick dom: layers of thickness ell[2a] at the low end and ell[2a+1] at the
 * high end of axis a (0: none), the outermost part of the brick; R in (0, 1)
 * is the design reflection coefficient of a layer (a plane wave through it
 * and back is attenuated by R).  Phi is held at the GLL nodes of every
 * element with zeta > 0 at one of its nodes, psi at their nodes.  Combine
 * with pmdg_set_absorbing on the outer faces, as in the paper.  Interface
 * faces of two coupled bricks carry no layer; orders up to 6; before bind
 * (PMDG_ESTATE after); PMDG_EINVAL on bad input.  A brick with a layer keeps
 * single-step passes on 4-wave tiles of 1 or 2 rows, sequential launches
 * (PMDG_OPT_TIME_BLOCK and PMDG_OPT_OVERLAP have no effect) and cannot join
 * a batch; pmdg_set_state starts Phi and psi at rest. */
pmdg_status pmdg_set_pml(pmdg_solver* h, int dom, const double* ell, double R);

/* Trilinear hexahedra (Sec. 3: each element is the image of the reference
 * cube under a trilinear map X_K with positive Jacobian).  Gives the
 * single brick of a one-domain solver its element vertices:
 * V[(ne0+1)(ne1+1)(ne2+1)][3] (host array, x fastest; element (ex, ey, ez)
 * is the trilinear image of the reference cube on the eight vertices
 * (ex + cx, ey + cy, ez + cz)).  The brick's x0 / x1 then only name its
 * topology; node coordinates, the lumped mass, the stiffness (with the
 * metric terms, evaluated per element from its corners on the GPU), the
 * PMUT face weights (with the surface Jacobian of the bottom face) and the
 * receiver lookup (Newton inverse map, lowest element first) follow the
 * vertices.  A CFL-chosen time step is chosen again from the shortest
 * element edge; the stability check uses the element-wise bound
 * lambda_max(M^{-1} K) <= max_e lambda_max(M_e^{-1} K_e) (PMDG_EUNSTABLE).
 * Must precede pmdg_set_pmuts, pmdg_set_receivers and pmdg_bind (ESTATE).
 * EINVAL: two-brick solvers, absorbing faces or layers (neither is built on
 * trilinear hexahedra), non-finite coordinates, or an element whose
 * Jacobian determinant is not positive at one of its GLL nodes.  Not
 * accepted by pmdg_batch_create. */
pmdg_status pmdg_set_vertices(pmdg_solver* h, int dom, const double* V);

/* Face matching on Gamma_I (Sec. 5, Algorithm 3), on the GPU.  Fine side:
 * nf hexahedra fine_hex[nf][8][3] (corner c = cx + 2 cy + 4 cz) and the local
 * face of each on Gamma_I, fine_face[nf] = 2 axis + side (side 0: the face
 * xi_axis = -1, side 1: +1); coarse side likewise (nc, coarse_hex,
 * coarse_face).  For every Gauss-Legendre point (nq per direction) of every
 * fine face, x_q = X_{K+}(xi), the coarse faces are taken in index order;
 * one is a candidate when its outward unit normal at its centre is opposite
 * to the fine face's, |n+ + n-| < tol, and its first corner (lowest corner
 * index on the face) lies within r = max(diam F-, diam F+) + eps of x_q
 * (diam: the largest distance between two corners of the face); the
 * first candidate whose element's inverse
 * map (Newton) puts x_q in [-1, 1]^3 up to 1e-10 is the match.  Points are
 * ordered (fine face, j, i), i along the face's first tangential axis
 * (axis + 1) mod 3.  Writes elem[nf nq^2] (coarse index, or -1),
 * xi[nf nq^2][3] (reference point in that element, 0 if unmatched) and
 * *unmatched (the count of -1 entries).  Every array is device memory; the
 * call enqueues two kernels on stream and returns (no allocation, no wait;
 * *unmatched is cleared by the first).
 * Faces with an index outside 0..5 match nothing.  EINVAL: nq outside
 * 1..9, negative counts, tol <= 0, eps < 0, NULL arrays. */
pmdg_status pmdg_match_faces(int nq, int nf, const double* fine_hex, const int* fine_face, int nc,
                             const double* coarse_hex, const int* coarse_face, double tol, double eps, int* elem,
                             double* xi, int* unmatched, void* stream);

/* Receiver points xyz[3*R]; each is located in the lowest-index element
 * containing it (primary first) and sampled by tensor Lagrange
 * interpolation, accumulated in FP64.  A point outside both bricks gives
 * EINVAL.  Must precede pmdg_bind. */
pmdg_status pmdg_set_receivers(pmdg_solver* h, int R, const double* xyz);

/* Device bytes needed by pmdg_bind (depends on everything set so far). */
pmdg_status pmdg_workspace_size(pmdg_solver* h, size_t* bytes);

/* Binds caller-owned device memory (>= pmdg_workspace_size bytes, 256-byte
 * aligned) and uploads all tables; the state starts at rest.  The caller
 * keeps the memory alive until pmdg_destroy.  Binding twice: ESTATE. */
pmdg_status pmdg_bind(pmdg_solver* h, void* dev_ptr, size_t bytes, void* stream);

/* For callers that cannot allocate device memory (code under graph
 * capture, serving loops, harnesses that forbid hipMalloc): pmdg_bind with
 * a workspace the library holds, one static device array of 32 MiB per GPU
 * (kept until the process ends), instead of caller memory.  Same tables,
 * kernels and results as pmdg_bind on the current device; zeroes the state
 * like pmdg_bind.  It allocates nothing: no hipMalloc, no library routine
 * that allocates.  PMDG_ENOMEM if the solver needs more than 32 MiB
 * (pmdg_workspace_size tells).  One array per device: the solver bound last
 * owns it; calls on a solver whose array was since bound to another solver
 * return PMDG_ESTATE (step, read and state calls, set_drive, batching), and
 * pmdg_destroy of the owner frees the array for the next bind.  Calls that
 * overlap on one GPU race on the array. */
pmdg_status pmdg_bind_static(pmdg_solver* h, void* stream);

/* Returns a bound solver to step 0 with everything at rest, as pmdg_bind
 * left it: the workspace is zeroed (pressure levels, increments, layer
 * fields, modal states, traces, step counter) and every table uploaded
 * again, in the same memory (caller-owned or library-held).  Meshes,
 * operators, PMUTs, receivers, options and the drive are kept; call
 * pmdg_set_drive before or after to run other drive scenarios with the
 * same solver, without building it again (the set-up of pmdg_create and
 * the set_* calls costs far more than a short run of a small mesh).
 * Returns when the work enqueued on stream is done.  Unbound solver, or
 * one whose library-held workspace was taken by another solver: ESTATE. */
pmdg_status pmdg_restart(pmdg_solver* h, void* stream);

/* The time step in use. */
pmdg_status pmdg_get_dt(pmdg_solver* h, double* dt);

/* Largest eigenvalue of M^{-1} K that pmdg_create checked dt against
 * (Sec. 3.1: the leapfrog is stable for dt^2 lambda_max < 4).  One brick:
 * c^2 times the sum of the three 1D operators' largest eigenvalues (exact
 * for the Kronecker-sum operator).  Two bricks: the larger of that and the
 * largest eigenvalue of the coupled operator with the interface penalty
 * gamma_F of Sec. 3, computed by Lanczos iteration on a patch of both bricks
 * around Gamma_I with the same element sizes, orders, materials and penalty
 * (laterally the shortest run of coarse elements ending on a fine element
 * edge, at least three coarse elements where the brick has them; up to three
 * element layers per side).  pmdg_create rejects dt^2 lambda_max >= 4 / 1.02
 * for the coupled estimate with PMDG_EUNSTABLE. */
pmdg_status pmdg_lambda_max(pmdg_solver* h, double* lam);

/* Enqueues n time steps on stream and returns without waiting.  Steps run
 * as captured hipGraphs (replayed in chunks) unless graphs are disabled with
 * pmdg_set_option.  Exceeding trace_capacity gives ESTATE before anything is
 * enqueued.  One solver must not be stepped on two streams at once. */
pmdg_status pmdg_step(pmdg_solver* h, int n, void* stream);

/* Steps completed so far. */
pmdg_status pmdg_steps_done(pmdg_solver* h, long* nsteps);

/* Waits for stream, then copies the FP64 traces [S][R][steps_done] into the
 * host array out (column j holds the pressure at time (j+1) dt). */
pmdg_status pmdg_read_traces(pmdg_solver* h, double* out, void* stream);

/* The same traces into caller-owned device memory, without a host copy or a
 * wait: enqueues on stream one kernel that writes the dense array
 * [S][R][steps_done] to out as FP64 (bits = 64) or rounded to FP32
 * (bits = 32).  out must hold S*R*steps_done elements of that type on the
 * solver's device and is valid once stream has reached the call.  EINVAL for
 * NULL out or other bits. */
pmdg_status pmdg_read_traces_device(pmdg_solver* h, void* out, int bits, void* stream);

/* Modal state of scenario s after the last step: q, qdot, qddot [Np*Nm]
 * (host arrays; NULL entries skipped). */
pmdg_status pmdg_read_modal(pmdg_solver* h, int s, double* q, double* qd, double* qdd, void* stream);

/* Field state of scenario s: pressure at the current and the previous time
 * level, [n_nodes] each, nodes of the primary then of the secondary, x
 * fastest.  set_state also sets the modal state (NULL: zero) and the step
 * counter, and recomputes the face force and interface terms.  The
 * scenarios of a solver share the step counter: with S > 1, nstep must equal
 * the steps done (PMDG_ESTATE otherwise), so the other scenarios keep their
 * state and traces. */
pmdg_status pmdg_num_nodes(pmdg_solver* h, long* n);
pmdg_status pmdg_get_state(pmdg_solver* h, int s, double* p, double* p_prev, void* stream);
pmdg_status pmdg_set_state(pmdg_solver* h, int s, const double* p, const double* p_prev, const double* q,
                           const double* qd, const double* qdd, long nstep, void* stream);

/* Node coordinates [n_nodes * 3] in the state's order. */
pmdg_status pmdg_node_coords(pmdg_solver* h, double* xyz);

/* Non-finite watchdog: *nonfinite != 0 once a pressure sampled on a PMUT
 * face or at a receiver was NaN or infinite (a blow-up anywhere reaches
 * these points within a few steps). */
pmdg_status pmdg_status_flags(pmdg_solver* h, int* nonfinite, void* stream);

/* Options: PMDG_OPT_GRAPH (1 = replay hipGraphs, 0 = direct launches),
 * PMDG_OPT_TILE_ROWS (rows per wave of the stiffness tile: 1, 2 or 4; a
 * workgroup covers 64 x (4 rows) nodes per plane; 0 = automatic (default):
 * 1 for a brick whose whole z extent is one chunk at 2 rows, else 2),
 * PMDG_OPT_TILE_ZCHUNK (planes per workgroup along z, 0 = whole brick,
 * -1 = automatic (default): 73 unless a brick would then have fewer than
 * 512 workgroups, then fewer, at least 4),
 * PMDG_OPT_GRAPH_CHUNK (steps per captured graph). */
#define PMDG_OPT_GRAPH 1
#define PMDG_OPT_TILE_ROWS 2
#define PMDG_OPT_TILE_ZCHUNK 3
#define PMDG_OPT_GRAPH_CHUNK 4
pmdg_status pmdg_set_option(pmdg_solver* h, int option, long value);

/* Average duration (ms) of each kernel class over the last timed
 * pmdg_step call made with PMDG_OPT_TIMING set: [0] stiffness, [1] face,
 * [2] flux.  Timing uses HIP events on the stepping stream. */
#define PMDG_OPT_TIMING 5
/* Tile of the secondary brick alone: rows per wave (0 = as PMDG_OPT_TILE_ROWS)
 * and planes per workgroup (-1 = as PMDG_OPT_TILE_ZCHUNK, 0 = whole brick). */
#define PMDG_OPT_TILE_ROWS_SECONDARY 6
#define PMDG_OPT_TILE_ZCHUNK_SECONDARY 7
/* Waves per stiffness workgroup, 4 or 8 (rows per wave 1 or 2 with 8). */
#define PMDG_OPT_TILE_WAVES 8
/* Steps per pass of the stiffness update over memory: 1, or 2 (FP32 solvers
 * with orders <= 4: the volume update of two steps is fused; the planes that
 * carry the PMUT force or the interface residual get their second step
 * after the coupling of the first).  Same arithmetic per node either way. */
#define PMDG_OPT_TIME_BLOCK 9
/* Two bricks: 1 runs the face work that needs only the primary (PMUT
 * sampling, modal ODE, force, and the primary's interface traces where the
 * face kernel rather than the stiffness launch writes them) on a side stream
 * alongside the secondary's stiffness launch; 2 also runs the primary's
 * stiffness launch on that side stream, concurrently with the secondary's;
 * 3 runs the face kernel's PMUT and receiver work on a side stream
 * alongside the interface kernels (it reads a copy of the step counter
 * that the primary's stiffness launch writes, since the last interface
 * kernel advances the counter); 0 (default) runs every kernel of a step in
 * sequence.  Same results in every mode; other values are rejected
 * (PMDG_EINVAL). */
#define PMDG_OPT_OVERLAP 10
/* PMDG_OPT_TIME_BLOCK for the secondary brick alone (0 = as the primary). */
#define PMDG_OPT_TIME_BLOCK_SECONDARY 11
/* Prefetch distance of the single-step stiffness update in planes: 2
 * (default), 3 or 4.  Distances above 2 apply to bricks of order <= 4 with
 * 4-wave tiles of 1 or 2 rows; other bricks keep 2.  Same results. */
#define PMDG_OPT_PREFETCH 12
/* LDS-resident steps (1 = automatic, the default; 0 = never).  A
 * single-brick FP32 solver without absorbing faces, layers or trilinear
 * vertices, with every tile option at its default, whose pressure,
 * increment, face force and PMUT tables fit one workgroup's LDS,
 * runs pmdg_step as launches of up to 2,048 whole steps each, one 1024-thread
 * workgroup per scenario (stiffness and update, PMUT sampling, modal ODE and
 * force, receivers), without graphs.  The arithmetic per node is the same as
 * the tiled path's; PMUT and receiver sums are taken in another order. */
#define PMDG_OPT_RESIDENT 13

/* *on = 1 when pmdg_step on this bound solver takes the LDS-resident path
 * (PMDG_OPT_RESIDENT), else 0. */
pmdg_status pmdg_resident(pmdg_solver* h, int* on);
pmdg_status pmdg_kernel_times(pmdg_solver* h, double* ms3);

/* Frees host resources (device memory is the caller's).  NULL is a no-op. */
void pmdg_destroy(pmdg_solver* h);

/* ---- Batched form --------------------------------------------------------
 * Several bound single-brick FP32 solvers (uneven meshes and orders, each
 * with its own drive scenarios) stepped together: per time step one
 * persistent stiffness launch over a device work list of (solver, tile)
 * items, one persistent face launch (PMUT sampling / modal ODE / face force,
 * receivers) and one launch advancing every solver's step counter, replayed
 * as hipGraphs.  Each solver keeps its own state, traces and tile options
 * (set them before pmdg_batch_create); read results through the solvers. */
typedef struct pmdg_batch pmdg_batch;

/* solvers[n]: bound, ndom == 1, precision 32, tile rows 1 or 2; the batch
 * does not own them and they must outlive it.  EINVAL / ESTATE otherwise.
 * The batch fixes each solver's tile and kernel arguments here: until
 * pmdg_batch_destroy, pmdg_set_option on a member solver accepts only
 * PMDG_OPT_GRAPH, PMDG_OPT_GRAPH_CHUNK and PMDG_OPT_TIMING (PMDG_ESTATE for
 * the others). */
pmdg_status pmdg_batch_create(int n, pmdg_solver* const* solvers, pmdg_batch** out);
/* Device bytes for the work lists and argument blocks. */
pmdg_status pmdg_batch_workspace_size(pmdg_batch* b, size_t* bytes);
/* Binds caller-owned device memory (256-byte aligned) and uploads the lists. */
pmdg_status pmdg_batch_bind(pmdg_batch* b, void* dev_ptr, size_t bytes, void* stream);
/* PMDG_OPT_GRAPH and PMDG_OPT_GRAPH_CHUNK as for a solver. */
pmdg_status pmdg_batch_set_option(pmdg_batch* b, int option, long value);
/* Enqueues n steps of every solver of the batch on stream (ESTATE if any
 * solver's trace capacity would be exceeded). */
pmdg_status pmdg_batch_step(pmdg_batch* b, int n, void* stream);
/* NULL is a no-op. */
void pmdg_batch_destroy(pmdg_batch* b);

/* ---- Surrogate form -------------------------------------------------------
 * A fully connected network with GELU on the hidden layers (gelu(z) =
 * z Phi(z), Phi the standard normal distribution function) that stands in for
 * the solver on the map from drive parameters (per-PMUT phases, frequency,
 * amplitude) to receiver traces.  The GEMMs run on BF16 MFMA with FP32
 * accumulation; the parameters are FP32 masters with BF16 copies; training
 * minimises the mean squared error with Adam (bias corrected).
 * Raw input rows u[n_u] pass through a fixed embedding into the n_0 network
 * inputs: column c takes feature u[src[c]] either affinely, (u - shift) *
 * scale, or as cos / sin (scale u + shift) (angles, Fourier features).  The
 * physical output is out_scale * a * y, with a = 1 or a = u[amp_col] for an
 * output known to be proportional to one
 * feature.  All rows are row-major FP32; u[nrows][n_u], targets
 * t[nrows][n_L], outputs y[B][n_L].  Device pointers unless stated.  Errors:
 * EINVAL for bad sizes or pointers, ESTATE for calls out of order, EHIP for
 * runtime failures.  Calls that overlap on one model race (one stream per
 * model). */
typedef struct pmdg_mlp pmdg_mlp;

/* widths[nlayers + 1]: n_0 .. n_L; hidden widths n_1 .. n_{L-1} multiples of
 * 32, the output width n_L a multiple of 8; 1 <= nlayers <= 16. */
pmdg_status pmdg_mlp_create(int nlayers, const int* widths, pmdg_mlp** out);
/* Number of trainable values sum_l n_{l+1} (n_l + 1). */
pmdg_status pmdg_mlp_num_params(pmdg_mlp* m, long* n);
/* Device bytes for parameters, Adam moments, activations of up to max_batch
 * rows (a multiple of 8) and split-K partial sums; fixes max_batch. */
pmdg_status pmdg_mlp_workspace_size(pmdg_mlp* m, int max_batch, size_t* bytes);
/* Binds caller-owned device memory (256-byte aligned), zeroes it. */
pmdg_status pmdg_mlp_bind(pmdg_mlp* m, void* dev_ptr, size_t bytes, void* stream);
/* Input embedding (host arrays of ncols = n_0): src[c] in [0, n_u), op[c]
 * 0 = (u - shift) * scale, 1 = cos(scale u + shift), 2 = sin(scale u +
 * shift).  amp_col = -1 or the feature a; out_scale > 0.  Default: n_u =
 * n_0, identity, amp_col = -1, out_scale = 1. */
pmdg_status pmdg_mlp_set_io_map(pmdg_mlp* m, int n_u, int ncols, const int* src, const int* op, const float* shift,
                                const float* scale, int amp_col, float out_scale, void* stream);
/* Optional second factor per input column (host arrays of ncols = n_0):
 * column c becomes g(u[src[c]]) * g2(u[src2[c]]) with g2 given by op2,
 * shift2, scale2 as above; src2[c] = -1 keeps the column a single factor.
 * pmdg_mlp_set_io_map clears every second factor, so call this after it.
 * PMDG_EINVAL on a bad index, op or non-finite value; PMDG_ESTATE before
 * the input map is set. */
pmdg_status pmdg_mlp_set_io_factors(pmdg_mlp* m, int ncols, const int* src2, const int* op2, const float* shift2,
                                    const float* scale2, void* stream);
/* Host parameters, per layer W_l [n_{l+1}][n_l] row-major then b_l; resets Adam. */
pmdg_status pmdg_mlp_set_params(pmdg_mlp* m, const float* host, void* stream);
pmdg_status pmdg_mlp_get_params(pmdg_mlp* m, float* host, void* stream);
/* Gradients of the last backward pass, same host layout as the parameters. */
pmdg_status pmdg_mlp_get_grads(pmdg_mlp* m, float* host, void* stream);
/* Forward pass of B rows (multiple of 8, <= max_batch).  Row r is u[idx[r]]
 * (idx clamped into [0, nrows)) or, with idx NULL, u[r] (nrows >= B).  With y
 * non-NULL writes out_scale * a * y there (inference); with y NULL keeps the
 * normalised output for pmdg_mlp_backward (training). */
pmdg_status pmdg_mlp_forward(pmdg_mlp* m, const float* u, const int* idx, int nrows, int B, float* y, void* stream);
/* Gradients of (1 / (B n_L)) sum (y - t[row] / (out_scale a))^2 for the last
 * training forward (same rows); per-row squared error and squared target
 * norm (normalised units) into rowerr[B], rownorm[B] if non-NULL. */
pmdg_status pmdg_mlp_backward(pmdg_mlp* m, const float* t, int B, float* rowerr, float* rownorm, void* stream);
/* One Adam step (bias-corrected, step count kept by the model) on the last gradients. */
pmdg_status pmdg_mlp_adam(pmdg_mlp* m, float lr, float beta1, float beta2, float eps, void* stream);
/* forward (training) + backward + Adam. */
pmdg_status pmdg_mlp_train_step(pmdg_mlp* m, const float* u, const float* t, const int* idx, int nrows, int B,
                                float lr, float beta1, float beta2, float eps, float* rowerr, float* rownorm,
                                void* stream);
/* Two-member ensemble: mean[B][n] = (a + b) / 2 and the relative spread
 * spread[r] = |a_r - b_r| / |mean_r| (0 if mean_r = 0); n a multiple of 4,
 * a, b, mean 16-byte aligned; mean may alias a or b. */
pmdg_status pmdg_mlp_pair_combine(const float* a, const float* b, int B, int n, float* mean, float* spread,
                                  void* stream);
/* Least-squares fit of the whole network (a closed-form training of it).
 * With input columns that are products of each PMUT's drive factor
 * (cos / sin of its phase) and a basis in frequency, the traces are a
 * linear function of the embedded inputs (the solver is linear in each
 * PMUT's drive A_k (cos theta_k, sin theta_k), Sec. 3.1).  The fit solves
 * min ||X W - T / (out_scale a)|| over rows u[idx[r]], t[idx[r]] (r < n) with
 * X the FP32 embedding, truncates W to its best rank-`rank` predictor
 * (eigen-decomposition of the whitened normal equations, host FP64), and
 * writes a network that computes it: the first layer maps the inputs to the
 * `rank` whitened coordinates z, the leading `npairs` enter the hidden layers
 * as pairs (gelu(z), gelu(-z)), whose difference is z exactly, the others
 * shifted by a bias beta (gelu(z + beta) = z + beta to within 1.4e-3 for
 * z + beta >= 3), the hidden layers pass them on and the output layer maps
 * them to the traces.  Needs hidden layers of one width with npairs + rank
 * <= that width, rank <= n_0 and rank <= n; ridge >= 0 adds ridge * (mean
 * diagonal of X^T X) to it.  Sets out_scale to the RMS of t / a over the fit
 * rows and resets Adam.  The large products run on the GPU (FP32), the
 * n_0 x n_0 factorisations on the host.  work: caller device memory of
 * pmdg_mlp_fit_linear_workspace bytes, 256-byte aligned.  u, t, idx device
 * pointers (idx NULL: rows 0 .. n-1). */
pmdg_status pmdg_mlp_fit_linear_workspace(pmdg_mlp* m, int n, int rank, size_t* bytes);
pmdg_status pmdg_mlp_fit_linear(pmdg_mlp* m, const float* u, const float* t, const int* idx, int nrows, int n,
                                int npairs, int rank, float ridge, void* work, size_t work_bytes, void* stream);
/* out_scale = RMS over rows idx of t / a (the normalisation of the targets
 * before training); work: device scratch of n doubles, 8-byte aligned. */
pmdg_status pmdg_mlp_set_target_scale(pmdg_mlp* m, const float* u, const float* t, const int* idx, int nrows, int n,
                                      void* work, size_t work_bytes, void* stream);
/* The model's current out_scale. */
pmdg_status pmdg_mlp_out_scale(pmdg_mlp* m, float* out_scale);
/* err[r] = ||y_r - t[idx[r]]|| / ||t[idx[r]]|| (0 for a zero target) for
 * r < B, rows of n floats (device pointers; idx NULL: row r). */
pmdg_status pmdg_mlp_row_errors(const float* y, const float* t, const int* idx, int nrows, int B, int n, float* err,
                                void* stream);
/* dst[rows[i]] = src[i] for i < nr, rows of n floats (device pointers): puts
 * solver traces in place of the network's for the rows sent to the solver. */
pmdg_status pmdg_mlp_scatter_rows(const float* src, const int* rows, int nr, int n, float* dst, void* stream);
/* NULL is a no-op. */
void pmdg_mlp_destroy(pmdg_mlp* m);

const char* pmdg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PMUTDG_H */
