/*
 * dg.h -- C ABI of the MI355X nodal discontinuous-Galerkin Euler library.
 *
 * The library integrates the three-dimensional compressible Euler equations
 * (Section 2.1, Eqs. 1-2) on a tetrahedral partition of the domain
 * (Appendix A, Eq. 9) with a nodal DG discretization of the weak form
 * (Appendix A, Eqs. 10-11), the local Lax-Friedrichs flux (Section 1.1) and a
 * five-stage fourth-order low-storage Runge-Kutta scheme for the resulting
 * ODE system dc/dt = f(c) (Appendix A, Eq. 12).  Boundary faces take the
 * pass-through state (Section 2.2), a characteristic outflow state, the
 * reflective wall (Section 2.3, Eq. 4), the mouthpiece inflow pulse
 * (Section 2.4, Eqs. 5-7) or a learned closure.
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every call returns int: DG_OK (0) or a negative DG_E* code; the message
 *   of the last failure is available from dg_last_error(ctx) (or
 *   dg_last_error(NULL) when no context could be created).
 * - "host" pointers are ordinary CPU memory, read during the call only;
 *   "device" pointers are GPU global memory (hipMalloc or torch tensors)
 *   owned by the caller, 16-byte aligned, never retained after the call.
 * - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *   Device work is enqueued asynchronously on it unless a call says
 *   otherwise.  Calls on one context must not overlap in time; a context is
 *   not safe for concurrent host threads.
 * - State layout: FP32 [K][5][Np], element-major, variables in the order
 *   (rho, rho u, rho v, rho w, E), nodes in the library's own order (use
 *   dg_nodes for their coordinates).  The stored values are the PERTURBATION
 *   of the conserved variables about the ambient state set at setup,
 *   q' = q - q0; the right-hand side of q' equals that of q.
 */
#ifndef DG_H
#define DG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------ */
#define DG_OK 0
#define DG_EINVAL (-1)    /* bad argument (null pointer, N, K, tag, flag)      */
#define DG_EMESH (-2)     /* invalid mesh (degenerate element, bad face match)  */
#define DG_ENOMEM (-3)    /* host or device allocation failed                  */
#define DG_EHIP (-4)      /* a HIP runtime call failed                         */
#define DG_ENONPHYS (-5)  /* rho <= 0, p <= 0 or NaN reached during dg_run     */
#define DG_ENODEV (-6)    /* device call on a context created host-only        */

/* ---- boundary tags (per element face) ---------------------------------- */
#define DG_BC_INTERIOR 0     /* matched to a neighbour                          */
#define DG_BC_OUTFLOW_CHAR 1 /* incoming acoustic characteristic set to ambient */
#define DG_BC_PASSTHRU 2     /* ghost = ambient rest state (Section 2.2)        */
#define DG_BC_WALL 3         /* slip wall, v - 2(v.n)n (Section 2.3, Eq. 4)      */
#define DG_BC_INFLOW 4       /* mouthpiece pulse (Section 2.4, Eqs. 5-7)         */
#define DG_BC_LEARNED 5      /* learned closure; characteristic outflow when no
                                network is attached                            */

/* ---- precision forms ---------------------------------------------------- */
#define DG_FP32 0        /* FP32 state, fluxes and contractions              */
#define DG_SPLIT_BF16 1  /* volume contraction as three BF16 MFMA products
                            (hi*hi + hi*lo + lo*hi), FP32 accumulation       */

/* ---- setup flags -------------------------------------------------------- */
#define DG_SETUP_HOST_ONLY 1 /* build host data only (no GPU needed); device
                                calls then return DG_ENODEV                  */
#define DG_SETUP_QUADRATURE 2 /* the paper's own discretization (Appendix A):
                                the weak form integrated with Gauss quadrature
                                exact to degree 2N in the volume and 2N + 1
                                on the faces (instead of the nodal strong form),
                                advanced by a two-stage second-order
                                Runge-Kutta scheme (SSP form) instead of
                                LSERK4; N = 1 or 2, FP32 form.  Same state
                                layout (nodal values of the order-N nodes, the
                                same polynomial space).  dg_rhs, dg_step
                                (one RK2 step; res unused), dg_run,
                                dg_run_fixed, dg_run_probes and the probes
                                apply; dg_stage, dg_set_kernel(1),
                                dg_set_damping, the learned closure and
                                batches do not (DG_EINVAL); dg_autotune
                                returns at once with blocks_per_cu = 0.      */

typedef struct dg_ctx dg_ctx;

/*
 * Mesh and problem description for dg_mesh_setup.
 *
 * N        polynomial order, 1..5.
 * K        number of tetrahedra, > 0.
 * xyz      host double [K][4][3]: coordinates of each element's vertices.
 * EToV     host int64 [K][4]: topological vertex ids; two faces are the same
 *          face when their id triples agree (periodic images share ids).
 * bc       host int8 [K][4]: tag of local face f, with f0={v0,v1,v2},
 *          f1={v0,v1,v3}, f2={v1,v2,v3}, f3={v0,v2,v3}.  A face listed by two
 *          elements is interior when both tags are DG_BC_INTERIOR and a
 *          two-sided boundary (zero-thickness wall) when both are non-zero.
 * gamma, rho0, u0, p0   ideal-gas ratio and ambient state (Section 2.2,
 *          Eq. 3 uses rho0 = 1.4, p0 = 1; any consistent scaling works).
 * inflow_amp, inflow_alpha   pulse p0 + amp (1 - cos(alpha t))/2 for
 *          0 <= t < 2 pi/alpha on DG_BC_INFLOW faces (Section 2.4).
 * precision  DG_FP32 or DG_SPLIT_BF16.
 * flags    0 or an OR of DG_SETUP_HOST_ONLY and DG_SETUP_QUADRATURE.
 */
typedef struct dg_mesh_desc {
  int32_t N;
  int32_t precision;
  int64_t K;
  const double* xyz;
  const int64_t* EToV;
  const int8_t* bc;
  double gamma;
  double rho0;
  double u0[3];
  double p0;
  double inflow_amp;
  double inflow_alpha;
  int32_t flags;
  int32_t reserved;
} dg_mesh_desc;

/*
 * Build a context: orientation fix (an element with negative Jacobian has
 * its local vertices 1 and 2 swapped, which exchanges the tags of faces 1
 * and 3), face matching, nodes, reference operators and affine geometry in
 * FP64 (Appendix A, Eqs. 9-11), then upload to the current HIP device.
 * Synchronous.  Host arrays are copied.  Errors: DG_EINVAL, DG_EMESH,
 * DG_ENOMEM, DG_EHIP; *out is NULL on failure.  Largest mesh: K x 5 x Np
 * values (and learned faces x 5 x Np) at most 2^31 - 1, i.e. 12,271,335
 * elements at N = 4 and 7,669,584 at N = 5 (the stage kernel's state
 * offsets are 32-bit); larger meshes are rejected with DG_EINVAL.
 */
int dg_mesh_setup(const dg_mesh_desc* d, void* stream, dg_ctx** out);

/* Free a context and all device memory it owns.  NULL is accepted. */
int dg_destroy(dg_ctx* ctx);

/* Message of the last failure on ctx (or of the last failed setup when
 * ctx is NULL).  The string lives until the next call on the same ctx. */
const char* dg_last_error(const dg_ctx* ctx);

/* Sizes: nodes per element, nodes per face, elements. */
int dg_sizes(const dg_ctx* ctx, int32_t* Np, int32_t* Nfp, int64_t* K);

/* Physical coordinates of every node, host double [K][Np][3], in the
 * library's node order and after the orientation fix. */
int dg_nodes(const dg_ctx* ctx, double* xyz_out);

/*
 * Host copies of the setup products (FP64), for checking the setup against
 * an independent construction.  Any pointer may be NULL.
 *   rst     [Np][3]           reference node coordinates
 *   Dr,Ds,Dt [Np][Np]         nodal differentiation matrices
 *   LIFT    [Np][4*Nfp]       M^-1 times the face mass matrices
 *   Fmask   int32 [4][Nfp]    node index of each face node
 */
int dg_reference_operators(const dg_ctx* ctx, double* rst, double* Dr, double* Ds,
                           double* Dt, double* LIFT, int32_t* Fmask);

/*
 *   drst_dx [K][3][3]   d(r,s,t)/d(x,y,z) per element
 *   J       [K]         Jacobian determinant of the reference map
 *   nrm     [K][4][3]   outward unit normal of each face
 *   Fscale  [K][4]      surface-to-volume Jacobian ratio sJ/J
 *   mapP    int64 [K][4][Nfp]  k'*Np + node of the neighbour node at the
 *                       same point, or -1 on boundary faces
 */
int dg_geometry(const dg_ctx* ctx, double* drst_dx, double* J, double* nrm,
                double* Fscale, int64_t* mapP);

/*
 * f(q) of Appendix A, Eq. 12: rhs = -(Dr Fr + Ds Fs + Dt Ft)
 * + sum_f Fscale_f LIFT_f dF_f at time t (t enters through inflow faces).
 * q, rhs: device FP32 [K][5][Np] perturbation states (see conventions).
 * Asynchronous on stream; no allocation.
 * Interface note: q holds q' = q - q0, not the conserved q (and so do the
 * states of dg_step, dg_stage, dg_run and the batch): acoustic perturbations
 * of 1e-3 p0 and below keep their digits in FP32.
 */
int dg_rhs(dg_ctx* ctx, const float* q, float* rhs, double t, void* stream);

/*
 * One five-stage low-storage RK step of size dt starting at time t:
 * for i = 1..5: res = a_i res + dt f(q, t + c_i dt); q = q + b_i res.
 * q (in/out) and res (scratch, contents ignored on entry since a_1 = 0):
 * device FP32 [K][5][Np].  Asynchronous on stream; no allocation.
 */
int dg_step(dg_ctx* ctx, float* q, float* res, double t, double dt, void* stream);

/*
 * One fused low-storage RK stage at stage time t_stage:
 *   res = a res + dt f(q_in, t_stage);  q_out = q_in + b res.
 * With a == 0 the previous contents of res are not read.  q_in and q_out
 * must be distinct device buffers (neighbour traces are read from q_in
 * while q_out is written); all three are FP32 [K][5][Np].  This is the
 * kernel dg_step and dg_run are made of, exposed for custom integrators
 * and for timing.  Asynchronous on stream; no allocation.
 */
int dg_stage(dg_ctx* ctx, const float* q_in, float* q_out, float* res, double a, double b,
             double t_stage, double dt, void* stream);

/*
 * nsteps steps with dt = cfl / max over elements, faces and face nodes of
 * (N+1)^2/2 * Fscale * (|u| + c), recomputed on the device at the start of
 * every step from the interior face traces.  The step sequence is captured
 * once in a HIP graph and replayed.  *t_inout is the start time on entry and
 * the end time on return; *dt_last (may be NULL) receives the last dt.
 * Synchronizes the stream once at the end.  Returns DG_ENONPHYS when a
 * non-physical state (rho <= 0, p <= 0 or NaN in a face trace) was seen;
 * dg_last_step then gives the first such step and the state is that of the
 * end of the run.
 */
int dg_run(dg_ctx* ctx, float* q, float* res, int64_t nsteps, double cfl,
           double* t_inout, double* dt_last, void* stream);

/*
 * dg_run with a fixed time step: every step takes dt (> 0) instead of the
 * CFL rule, so that runs on different meshes advance in lockstep (used to
 * compare a truncated domain against a larger one).  Same ownership,
 * synchronization and errors as dg_run.
 */
int dg_run_fixed(dg_ctx* ctx, float* q, float* res, int64_t nsteps, double dt, double* t_inout,
                 void* stream);

/* Step index (0-based, within the last dg_run) of the first non-physical
 * state, or -1. */
int64_t dg_last_step(const dg_ctx* ctx);

/* dt of the CFL rule above for state q, written to *dt (host).
 * Synchronizes the stream. */
int dg_stable_dt(dg_ctx* ctx, const float* q, double cfl, double* dt, void* stream);

/*
 * Convert primitive fields (rho, u, v, w, p) at the nodes, device FP32
 * [K][5][Np] given as perturbations about the ambient state
 * (rho - rho0, u - u0, v - v0, w - w0, p - p0), into the conserved
 * perturbation state q' of the same layout (Eq. 2).
 */
int dg_prim_to_state(dg_ctx* ctx, const float* prim, float* q, void* stream);

/* Inverse of dg_prim_to_state. */
int dg_state_to_prim(dg_ctx* ctx, const float* q, float* prim, void* stream);

/* ---- batched ensembles ---------------------------------------------------
 * Several geometries (contexts created with the same N, gamma and ambient
 * state) times up to 16 members that differ by their inflow-pulse amplitude,
 * advanced together by one persistent stage kernel per RK stage, captured in
 * one HIP graph.  Member states are stored member-innermost:
 * FP32 [K_g][5][Np][16] per geometry g (slots >= members are ignored), as
 * perturbations about the ambient state like single states.
 */
typedef struct dg_batch dg_batch;

/* Bind ngeom contexts (borrowed: they must outlive the batch) with
 * `members` (1..16) members each.  Errors: DG_EINVAL on mismatched N or
 * physics, DG_ENOMEM, DG_EHIP. */
int dg_batch_create(dg_ctx* const* geoms, int ngeom, int members, void* stream,
                    dg_batch** out);

int dg_batch_destroy(dg_batch* b);

const char* dg_batch_last_error(const dg_batch* b);

/*
 * nsteps steps of every member, each with its own time step from the CFL
 * rule of dg_run and its own time.  q[g], res[g]: device FP32
 * [K_g][5][Np][16]; amps: host double [ngeom][16] inflow amplitudes;
 * t_inout: host double [ngeom][16] start times in, end times out.
 * Synchronizes once at the end.  Returns DG_ENONPHYS when any member met a
 * non-physical state (dg_batch_first_bad gives the steps).
 */
int dg_batch_run(dg_batch* b, float* const* q, float* const* res, const double* amps,
                 int64_t nsteps, double cfl, double* t_inout, void* stream);

/* First non-physical step per member in the last dg_batch_run, or -1:
 * host int64 [ngeom][16]. */
int dg_batch_first_bad(const dg_batch* b, int64_t* steps);

/* Launch shape of the batched stage kernel: resident blocks per CU
 * (0 = as many as fit) and wavefronts per block (1, 2, 4 or 8).  Used by
 * the autotuner; takes effect at the next dg_batch_run. */
int dg_batch_set_launch(dg_batch* b, int blocks_per_cu, int waves_per_block);

/* Resident stage blocks per CU of a single-solve context (0 = as many as
 * fit); used by the autotuner. */
int dg_set_launch(dg_ctx* ctx, int blocks_per_cu);

/* Stage kernel of a single-solve context: 0 = tile-cooperative (four
 * wavefronts share a 16-element tile and split the contraction), 1 =
 * role-specialized (per block, four surface wavefronts form the face jumps
 * of one tile while four contraction wavefronts, holding the operator in
 * registers, run the products and the RK update of the previous tile; FP32
 * form, N <= 4).  Same results up to floating-point summation order.  Used
 * by the autotuner; DG_EINVAL when the variant does not apply. */
int dg_set_kernel(dg_ctx* ctx, int variant);
int dg_get_kernel(const dg_ctx* ctx);

/* ---- launch-shape autotuner -------------------------------------------------
 * Times every launch shape of the stage kernel (resident blocks per CU, and
 * the stage-kernel variant where the role-specialized one applies; for
 * batches blocks per CU and wavefronts per block) on the caller's stream
 * with HIP events,
 * applies the fastest and appends it to the text cache at cache_path (NULL or
 * "" for no cache) under a key made of the workload sizes and the device
 * architecture and CU count; a cached entry is applied without timing.
 * Results of the solver do not depend on the launch shape.
 * q is read and left unchanged; res is overwritten (scratch).  The chosen
 * shape is returned through the optional out pointers.  Synchronizes.
 * Interface note: it times on a caller-given state and scratch buffer and
 * keeps a plain-text cache (not JSON), so that no hidden allocation occurs. */
int dg_autotune(dg_ctx* ctx, const float* q, float* res, const char* cache_path,
                int* blocks_per_cu, void* stream);

int dg_batch_autotune(dg_batch* b, float* const* q, float* const* res, const char* cache_path,
                      int* blocks_per_cu, int* waves_per_block, void* stream);

/* ---- learned boundary closure ------------------------------------------------
 * A multilayer perceptron 78 -> 128 -> 128 -> 75 with GELU activations maps a
 * boundary face's characteristic ghost (its interior trace with the incoming
 * acoustic characteristic removed) -- the perturbation q - q0 of the five
 * conserved variables at its 15 face nodes (N = 4), variable-major
 * x[v * 15 + i], divided by a scale -- followed by the face's outward unit
 * normal, to the exterior trace in the same scale.  It
 * stands in for the ghost state of the boundary conditions of Section 2
 * (faces tagged DG_BC_LEARNED), with the characteristic ghost as fallback.
 * The scale is a fixed amplitude norm > 0, or, with norm = 0, each face's
 * own largest |q - q0| over its input trace (inputs and outputs scale
 * together, so the learned map is amplitude-equivariant).
 * Parameters: one FP32 vector of DG_MLP_PARAMS values, W1 [128][78], b1,
 * W2 [128][128], b2, W3 [75][128], b3 (row-major, out x in).
 * Training: FP32, loss = mean over rows of |y_hat - y|^2 / (|y|^2 + 1e-6),
 * Adam (beta 0.9, 0.999, eps 1e-8).  Inference in the solver: BF16 weights
 * and activations with FP32 accumulation.
 */
#define DG_MLP_PARAMS 36299
typedef struct dg_mlp dg_mlp;

/* params: host FP32 [DG_MLP_PARAMS], copied.  Synchronizes.
 * Interface note: there is no seed argument; the library draws no random
 * numbers, so the initial weights always come from the caller. */
int dg_mlp_create(const float* params, void* stream, dg_mlp** out);
int dg_mlp_destroy(dg_mlp* m);
const char* dg_mlp_last_error(const dg_mlp* m);
/* host FP32 [DG_MLP_PARAMS]; synchronize */
int dg_mlp_get_params(dg_mlp* m, float* params, void* stream);
int dg_mlp_set_params(dg_mlp* m, const float* params, void* stream);

/* Y [B][75] = network(X [B][78]); device pointers; bf16 != 0 selects the
 * BF16 inference kernel, else FP32.  Asynchronous (FP32 may allocate its
 * workspace the first time a larger B is seen). */
int dg_mlp_infer(dg_mlp* m, const float* X, float* Y, int64_t B, int bf16, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the FP32
 * forward of dg_mlp_infer(m, X, Y, B, 0, stream), with the same kernels and
 * bitwise the same Y, whose hidden activations live in a fixed device array
 * of the library instead of a workspace it allocates.  The array holds
 * DG_MLP_NOALLOC_ROWS rows (4 x 128 FP32 each, 8 MiB in all); each GPU the
 * library runs on keeps its own copy until the process ends.  X [B][78],
 * Y [B][75]: device pointers on the current device (the one m was created
 * on), caller-owned; B = 0 does nothing and reads neither pointer.  Calls no
 * hipMalloc or hipFree.  Errors: DG_EINVAL for a null pointer (B > 0),
 * B < 0 or B > DG_MLP_NOALLOC_ROWS; DG_EHIP if the array's
 * address cannot be obtained or a launch fails.  Every call on one GPU shares
 * that GPU's array (nothing in it needs to start at zero; each call
 * overwrites what it reads): calls that overlap on one GPU, from two streams
 * or two host threads, race, and the caller must order them.  Asynchronous
 * on stream. */
#define DG_MLP_NOALLOC_ROWS 4096
int dg_mlp_infer_noalloc(dg_mlp* m, const float* X, float* Y, int64_t B, void* stream);

/* Loss and gradient for rows (X [B][78], Y [B][75]) (device): grads is a
 * device FP32 [DG_MLP_PARAMS] (NULL: internal); *loss (host, optional) is
 * read back with a synchronization.  Deterministic. */
int dg_mlp_grad(dg_mlp* m, const float* X, const float* Y, int64_t B, float* loss, float* grads,
                void* stream);

/* One Adam step on the minibatch rows[0..B) of the device data set
 * (X [n_rows][78], Y [n_rows][75]); rows is a device int64 array (indices
 * are clamped to the set), or NULL for the first B rows.  lr: step size.
 * *loss (host, optional) gets the minibatch loss before the update and
 * synchronizes. */
int dg_mlp_train_step(dg_mlp* m, const float* X, const float* Y, int64_t n_rows,
                      const int64_t* rows, int64_t B, float lr, float* loss, void* stream);

/* Attach (m != NULL) or detach (m == NULL) a network to the context's faces
 * tagged DG_BC_LEARNED (N = 4 only).  norm: the trace normalization (0: per
 * face, see above).  On a face whose interior trace has its largest |p'| in
 * [p_lo, p_hi] and whose network state has rho > 0 and p > 0 at every node,
 * the ghost is  char + blend * (network - char)  (blend in [0, 1]; 1 = the
 * network alone), elsewhere the characteristic ghost.  The network is
 * borrowed and must outlive the attachment; weight updates take effect at the
 * next launch.
 * Interface note: besides the amplitude window (p_lo, p_hi) it takes the
 * input normalization and the blend weight. */
int dg_set_learned_bc(dg_ctx* ctx, dg_mlp* m, double norm, double p_lo, double p_hi,
                      double blend);

/* Number of faces tagged DG_BC_LEARNED; when faces is not NULL, writes their
 * k * 4 + f (host int64) in the order the solver indexes them. */
int64_t dg_learned_faces(const dg_ctx* ctx, int64_t* faces);

/* Network rows from a state: for faces[j] = k * 4 + f (device int64 [nf]),
 * X[j] (device FP32 [nf][78]) = characteristic ghost of the interior trace /
 * scale and the normal, and when Y is not NULL, Y[j] (device [nf][75]) =
 * exterior trace / scale (scale = norm, or with norm = 0 the largest
 * |q - q0| of the face's characteristic ghost): the
 * neighbour's trace on interior faces (a larger domain's solution), the ghost
 * of the face's tag on boundary faces.  Face indices outside the mesh are
 * skipped.  Asynchronous.
 * Interface note: the extra norm argument selects the same normalization as
 * dg_set_learned_bc, so sampled rows match what the solver feeds the network. */
int dg_sample_traces(dg_ctx* ctx, const float* q, const int64_t* faces, int64_t nf, double norm,
                     float* X, float* Y, void* stream);

/* ---- absorbing layer ----------------------------------------------------
 * A sponge zone next to the outer boundary as a third closure beside the
 * characteristic and learned ghosts (the absorbing-layer treatments the
 * introduction surveys): every node relaxes towards the ambient state,
 *     dq'/dt = f(q') - sigma(x) q',
 * at a rate sigma(x) >= 0 the caller chooses (zero outside the layer,
 * ramping up towards the boundary).  sigma: device FP32 [K][Np] in the
 * library's node order (see dg_nodes), borrowed: it must stay valid while the
 * context uses it; NULL turns the layer off.  Applies to dg_rhs, dg_step,
 * dg_stage and the runs of this context (not to batches: dg_batch_create
 * rejects a context with a layer).  Both stage-kernel variants apply
 * it.  Errors:
 * DG_ENODEV on a host-only context. */
int dg_set_damping(dg_ctx* ctx, const float* sigma);

/* ---- curved (isoparametric) elements -----------------------------------
 * Section 3 ascribes the reflections of the spherical outer domain to its
 * boundary being built from flat faces; curved boundary elements are the
 * remedy it names.  xyz_nodes (host FP64 [K][Np][3], the library's node
 * order, see dg_nodes and dg_reference_operators) gives the physical
 * position of every node; each element's map becomes the degree-N
 * polynomial through its nodes.  Elements whose nodes lie within tol times
 * their longest edge of the straight-sided positions stay straight; for the
 * others ("curved") the library keeps, at every node, the metric terms
 * d(r,s,t)/d(x,y,z) of that map and, at every face node, the outward unit
 * normal and sJ/J, and evaluates their right-hand side as
 *   dq/dt(node n) = - sum_a sum_d (d r_a/d x_d)(n) (D_a F_d)(n)
 *                   + sum_f LIFT_f [ (sJ/J) dF ]_f,
 * (the volume term in chain-rule form, which is the straight-sided operator
 * when the metric terms are constant; dF the local Lax-Friedrichs jump with
 * each face node's own normal, one lambda per face).  The time-step rule
 * keeps each element's straight-sided Fscale.  Curved elements are computed
 * by a separate pass after the stage kernel, which leaves their outputs and
 * their share of the time-step rate to it, so the straight elements keep
 * the full-speed path.  Copies what it needs; the host array may be freed on
 * return.  NULL clears the curved set.  Applies to dg_rhs, dg_step,
 * dg_stage, the runs and dg_autotune of this context; dg_probe_setup,
 * called after it, locates points in curved elements by inverting their
 * maps (see there).  On a host-only context the curved set is checked and
 * kept for probe location only.
 * n_curved_out (may be NULL) receives the number of curved elements.
 * Errors: DG_EINVAL for tol <= 0, a context with the quadrature scheme or a
 * learned closure, a node Jacobian <= 0, or node positions that do not
 * coincide (to tol times the edge length) on a shared face; DG_ENOMEM /
 * DG_EHIP.  Any call first drops the
 * previous curved set, so after an error the context has none.
 * dg_batch_create and dg_set_learned_bc reject a context with curved
 * elements.  Synchronous. */
int dg_set_curved(dg_ctx* ctx, const double* xyz_nodes, double tol, int64_t* n_curved_out,
                  void* stream);

/* ---- pressure probes and spectra -----------------------------------------
 * Section 3 samples the pressure of each run at sensor points inside and
 * around the instrument and compares the frequency content of those signals
 * (amplitude spectra in dB) between domains.  A probe evaluates the
 * numerical solution itself at a point: the nodal polynomial of the element
 * containing the point, interpolated in the conserved perturbation q', then
 * p - p0 from it (Eq. 2). */

/* Locate n points (host double [n][3], physical coordinates) in the mesh
 * and keep them, with their nodal interpolation weights, as the context's
 * probe set (replacing any previous one).  A point on a face shared by two
 * elements belongs to the element whose smallest barycentric coordinate there
 * is largest (the first such element on ties).  elements_out (host int64
 * [n]) receives each point's element and weights_out (host double [n][Np])
 * its interpolation weights w (value at the point = sum_i w[i] u[node i], in
 * the library's node order); either may be NULL.  On a host-only context
 * the points are located and weighed but no probe set is kept.
 * With a curved set (dg_set_curved, set before), a point whose straight-sided
 * element is curved, or that lies outside the straight-sided mesh, is
 * located by inverting the maps of the curved elements near it: it belongs
 * to the one whose reference point has the largest smallest barycentric
 * coordinate, which must be >= -1e-9 (so a point between a chord and a face
 * bent outward is found, and one beyond a curved face that moved into its
 * straight-sided element goes to the neighbour whose curved image holds it).
 * Synchronous.  Errors: DG_EINVAL for n outside 1..2^20, a point outside
 * the mesh (tolerance 1e-9 in barycentric coordinates) or a curved map that
 * does not invert, DG_ENOMEM. */
int dg_probe_setup(dg_ctx* ctx, const double* xyz, int32_t n, int64_t* elements_out,
                   double* weights_out);

/* p - p0 at every probe of state q (device, the state layout) into out
 * (device FP32 [n]).  Asynchronous.  DG_EINVAL without probes. */
int dg_probe_sample(dg_ctx* ctx, const float* q, float* out, void* stream);

/* dg_run_fixed that also records, after every step j (0-based), p - p0 at
 * every probe into series[j][p] (device FP32 [nsteps][n], caller-owned): a
 * uniformly sampled signal with spacing dt.  Same ownership, synchronization
 * and errors as dg_run_fixed; DG_EINVAL without probes or with a null
 * series. */
int dg_run_probes(dg_ctx* ctx, float* q, float* res, int64_t nsteps, double dt, double* t_inout,
                  float* series, void* stream);

/* One-sided amplitude spectra of n_signals real signals of n_samples
 * uniformly spaced samples, series[j][s] (device FP32, the layout
 * dg_run_probes writes): db[s][k] (device FP32 [n_signals][n_samples/2 + 1])
 * = 20 log10(A_k / p_ref) with A_k = 2 |X_k| / n_samples (|X_k| / n_samples
 * at k = 0 and k = n_samples/2), X_k = sum_j x_j exp(-2 pi i k j / n_samples),
 * floored at -600 dB.  Bin k is the frequency k / (n_samples dt).  No
 * context; errors through dg_last_error(NULL).  Asynchronous.  DG_EINVAL for
 * n_samples < 2, n_signals outside 1..65535 or p_ref <= 0. */
int dg_spectrum(const float* series, int64_t n_samples, int32_t n_signals, double p_ref,
                float* db, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* DG_H */
