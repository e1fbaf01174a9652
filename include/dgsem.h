/*
 * dgsem.h -- C ABI of the MI355X (gfx950) split-form DGSEM Navier-Stokes operator.
 *
 * The library evaluates the semi-discrete right-hand side dU/dt = L(U) of the
 * compressible Navier-Stokes equations on an axis-aligned tensor-product mesh
 * of hexahedra with Legendre-Gauss-Lobatto (LGL) collocation (paper Sec. 2.2:
 * split-form DG on LGL nodes) and advances it with the five-stage fourth-order
 * low-storage Runge-Kutta scheme (paper Sec. 4).  The operator is:
 *   BR1 lifting of the primitive gradients grad(u, v, w, T);
 *   Kennedy-Gruber split-form flux-differencing volume integral;
 *   local Lax-Friedrichs surface flux (Kennedy-Gruber central part) and the
 *   BR1 central viscous surface flux, with periodic or isothermal no-slip
 *   wall boundaries (paper Sec. 3-4: periodic and wall boundaries, ideal gas,
 *   viscous fluxes);
 *   strong-form surface-to-volume lifting and the affine Jacobian scaling.
 *
 * Conventions shared by every call
 *   - A DOF is one collocation node of one element: n_dof = nx ny nz (N+1)^3.
 *   - State layout (all device pointers, float64, caller owned, contiguous):
 *       U[v][e][k][j][i],  v in (rho, rho u, rho v, rho w, E),
 *       e = ex + nx (ey + ny ez),  i is the x node index and runs fastest.
 *     A state therefore holds 5 n_dof doubles.
 *   - Gradient layout (dg_eval_lift): grad[3 q + d][e][k][j][i], q in (u, v, w, T),
 *     d in (x, y, z); 12 n_dof doubles.
 *   - Every call is asynchronous on the HIP stream given to dg_init_mesh and
 *     returns a dg_status; no exception crosses the ABI.  Device-side
 *     failures (non-positive density or pressure, NaN) are reported by dg_sync.
 *   - The library never allocates device memory: the caller provides the
 *     workspace (dg_workspace_bytes, dg_bind_workspace); the one exception is
 *     the static 64 MiB device array of dg_eval_rhs_noalloc, which exists per
 *     device with the loaded library.  A context is bound to one stream and
 *     one device and is not thread-safe.
 */
#ifndef DGSEM_H
#define DGSEM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DG_OK = 0,
  DG_EINVAL = 1,        /* invalid argument or mesh description                  */
  DG_ESTATE = 2,        /* call order violated (e.g. no workspace bound yet)     */
  DG_EHIP = 3,          /* a HIP runtime call failed (dg_last_error has the text) */
  DG_ENONPHYS = 4,      /* a kernel saw rho <= 0, p <= 0 or a NaN (from dg_sync) */
  DG_EUNSUPPORTED = 5   /* valid request that this library does not implement    */
} dg_status;

#define DG_BC_PERIODIC 0
#define DG_BC_ISOTHERMAL_WALL 1
#define DG_BC_WALL_MODEL 2   /* slip, adiabatic wall whose shear stress comes from the
                                algebraic wall model (dg_wall_stress) evaluated on the
                                state of every stage; FP64 or mixed; no adjoint       */

#define DG_FP64 0
#define DG_MIXED 1
#define DG_MIXED_NOREF 2  /* DG_MIXED without the reference-state subtraction (measurement) */

/* Convective fluxes (dg_physics.flux). */
#define DG_FLUX_KG_LLF 0  /* Kennedy-Gruber split-form volume flux; local Lax-Friedrichs
                             surface flux with the Kennedy-Gruber central part        */
#define DG_FLUX_EC_ROE 1  /* the paper's production pair (Sec. 4): Chandrashekar's
                             entropy-conserving volume flux; Roe surface flux with
                             Harten's entropy correction (Harten-Hyman form), its
                             central part the Chandrashekar flux.  DG_FP64, or
                             DG_MIXED (the volume flux in FP32 relative to each
                             element's reference state; DG_MIXED_NOREF gets
                             DG_EUNSUPPORTED); the adjoint covers it                   */

/* Viscosity laws (dg_physics.viscosity). */
#define DG_VISC_CONSTANT 0    /* mu constant                                              */
#define DG_VISC_SUTHERLAND 1  /* Sutherland's law, the paper's (Sec. 4) for its working
                                 fluid: mu(T) = mu (T / T_ref)^(3/2) (T_ref + S) / (T + S),
                                 mu being the viscosity at T_ref; T_ref and S in the units
                                 of T; taken at each node's temperature (at a wall: the
                                 interior face node's; in the wall model: the wall
                                 temperature's).  FP64 or mixed; the adjoint covers it    */

typedef struct dg_ctx dg_ctx;

/* Mesh description.  faces[d] are host arrays of nelem[d] + 1 strictly
 * increasing coordinates; they are copied by dg_init_mesh.  bc[d] applies to
 * both ends of direction d.  N must be 3, 5 or 7 (templated kernels).       */
typedef struct {
  int N;
  int nelem[3];
  const double* faces[3];
  int bc[3];
  double T_wall;      /* wall temperature of DG_BC_ISOTHERMAL_WALL ends          */
  int wm_node;        /* interface LGL node (1..N, from the wall) of the wall model
                         at DG_BC_WALL_MODEL ends; ignored otherwise            */
  const double* nodes;/* NULL: the axis-aligned elements of `faces`.  Otherwise
                         curved hexahedra (the paper's production meshes, Sec. 4):
                         host array of the physical node coordinates
                         nodes[(n nE + e) (N+1)^3 + node], n = x, y, z, e and node
                         in the state's canonical order, copied by dg_init_mesh;
                         each element is the degree-N interpolant of its nodes
                         (Kopriva's curl-form metric terms, contravariant
                         two-point fluxes with averaged metrics); the elements
                         keep the structured connectivity of nelem, periodic
                         or isothermal-wall ends (the wall normal is the face's
                         metric vector); faces may be NULL.  DG_FP64 or DG_MIXED
                         with either flux pair (the Roe flux along the face's
                         unit normal, scaled by its length); the wall model
                         and the adjoint, lifting or kinetic-energy calls give
                         DG_EUNSUPPORTED.  The workspace holds the metric
                         terms, 10 FP64 values per DOF (+ 10 FP32 values in
                         mixed precision) and the FP64 ones again per node
                         on the element boundary.  A non-positive Jacobian at any node
                         makes dg_bind_workspace fail with DG_EINVAL.          */
} dg_mesh_desc;

/* Gas and scheme switches.  The heat conductivity is
 * kappa(T) = mu(T) gamma R / ((gamma - 1) Pr).  The fields after `flux` may be
 * left zero (constant viscosity).                                            */
typedef struct {
  double gamma, R, mu, Pr;
  int viscous;        /* 0: Euler fluxes only (no lifting), 1: Navier-Stokes      */
  int precision;      /* DG_FP64, or DG_MIXED: FP32 lifting, volume fluxes,
                         line sums and Lax-Friedrichs surface fluxes; FP64
                         state, primitive recovery, lifting corrections, the
                         Roe surface flux and RK accumulation; p, e and T enter
                         the FP32 parts relative to a per-element reference
                         value (the surface fluxes as FP64 differences of the
                         two sides)                                            */
  int central_only;   /* 1: drop the surface dissipation (Lax-Friedrichs or Roe):
                         test switch                                             */
  int flux;           /* DG_FLUX_KG_LLF or DG_FLUX_EC_ROE                          */
  int viscosity;      /* DG_VISC_CONSTANT or DG_VISC_SUTHERLAND                     */
  double T_ref, S;    /* Sutherland's law: reference temperature (> 0) and
                         Sutherland's temperature (>= 0); ignored otherwise      */
} dg_physics;

/* Library version string (static storage). */
const char* dg_version(void);

/* LGL nodes xi[0..N] and weights w[0..N] (host arrays, caller owned), the
 * basis of the paper's Sec. 2.2 scheme.  Pure host computation, any N in 1..16. */
dg_status dg_lgl(int N, double* xi, double* w);

/* Validate the mesh and physics, build the host tables and create a context
 * on `hip_stream` (a hipStream_t, NULL = default stream).  No device work.
 * The mesh is the paper's element decomposition (Sec. 2.1-2.2: hexahedral
 * elements, each with (N+1)^3 LGL collocation nodes); the physics are the
 * ideal gas with viscous fluxes of Sec. 4 and the flux pairs above.  The
 * context copies everything it needs from `mesh` and `phys`; the caller keeps
 * ownership of both.  On error *out is left unchanged.
 * Errors: DG_EINVAL (null pointers, non-monotone faces, bad bc, gamma <= 1,
 * R <= 0, mu < 0, Pr <= 0, empty mesh, unknown precision, flux or viscosity
 * law, Sutherland's law with T_ref <= 0 or S < 0),
 * DG_EUNSUPPORTED (N not in {3, 5, 7}; DG_FLUX_EC_ROE, DG_BC_WALL_MODEL or
 * DG_VISC_SUTHERLAND with mixed precision).                                  */
dg_status dg_init_mesh(const dg_mesh_desc* mesh, const dg_physics* phys, void* hip_stream,
                       dg_ctx** out);

/* Bytes of device workspace the context needs.  with_adjoint != 0 adds the
 * buffers of the VJP calls.                                                  */
dg_status dg_workspace_bytes(const dg_ctx* ctx, int with_adjoint, size_t* bytes);

/* Number of DOFs (nodes) of the mesh. */
dg_status dg_n_dof(const dg_ctx* ctx, long long* n_dof);

/* Bind caller-owned device memory (>= dg_workspace_bytes, 256-byte aligned)
 * and upload the tables.  May be called again to rebind.                      */
dg_status dg_bind_workspace(dg_ctx* ctx, void* dev_ptr, size_t bytes, int with_adjoint);

/* Copy a state (layout above) into the context and clear the RK register:
 * the initial value U(t0) of the semi-discrete system dU/dt = L(U) (paper
 * Sec. 2.2) that dg_rk_step advances.  U_dev (device, 5 n_dof doubles, caller
 * owned) is read on the context's stream.  Errors: DG_EINVAL (null pointer),
 * DG_ESTATE (no workspace bound).                                            */
dg_status dg_set_state(dg_ctx* ctx, const double* U_dev);

/* Copy the context's current state (the RK solution of paper Sec. 4 after
 * the steps taken so far) to U_dev (device, 5 n_dof doubles, caller owned),
 * asynchronously on the context's stream.  Errors: DG_EINVAL, DG_ESTATE.   */
dg_status dg_get_state(const dg_ctx* ctx, double* U_dev);

/* Ut = L(U) (paper Sec. 2.2 semi-discrete operator).  U and Ut must not overlap.
 * t is the physical time (the operator has no time-dependent terms).       */
dg_status dg_eval_rhs(dg_ctx* ctx, const double* U_dev, double* Ut_dev, double t);

/* Allocation-free dg_eval_rhs, for callers that cannot allocate device
 * memory or bind a workspace (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Ut = L(U) by the same kernels in
 * the same order as dg_eval_rhs (bitwise the same result); the derivative
 * matrix, the element scale tables, the face viscous fluxes, the wall-model
 * stress and the status word live in a static device array of the library,
 * 64 MiB per device, instead of the workspace, and the call allocates
 * nothing.  The context needs no workspace (one from dg_init_mesh alone
 * works).  U and Ut: device arrays of 5 n_dof doubles in the state layout,
 * caller owned, not overlapping.  status_dev: a device int that a
 * non-physical state sets to 1 (the caller clears it), or NULL to drop that
 * report.  Every call on a device rewrites that device's array: calls that
 * overlap on one device race (one stream at a time).  Errors: DG_EINVAL (null
 * pointers; a mesh whose face fluxes and tables exceed the 64 MiB: at N = 7
 * about 5,400 elements in FP64, 10,900 in mixed precision), DG_EUNSUPPORTED
 * (curved elements), DG_EHIP.                                                */
dg_status dg_eval_rhs_noalloc(dg_ctx* ctx, const double* U_dev, double* Ut_dev, double t,
                              int* status_dev);

/* BR1 lifted gradients of (u, v, w, T) of U, layout above (FP64 contexts only). */
dg_status dg_eval_lift(dg_ctx* ctx, const double* U_dev, double* grad_dev);

/* Advance the context's state by nsteps steps of size dt of the five-stage
 * low-storage RK scheme (paper Sec. 4): per stage s, G <- A_s G + dt L(U),
 * U <- U + B_s G.  t is the time at the start.                               */
dg_status dg_rk_step(dg_ctx* ctx, double t, double dt, int nsteps);

/* dg_rk_step captured once into a HIP graph, for loops that launch-bound
 * (small meshes: 10 kernel launches per step).  dg_rk_graph_build records
 * nsteps (even, >= 2) steps of size dt on a private stream and instantiates
 * them; nothing runs and the state is unchanged.  dg_rk_graph_launch enqueues
 * the graph `repeats` times on the context's stream: each repeat advances the
 * state by nsteps steps exactly as dg_rk_step would (same kernels, same
 * order, bitwise the same result).  The graph holds the workspace pointers: a
 * new dg_bind_workspace or dg_rk_graph_build drops it, dg_free releases it.
 * Errors: DG_EINVAL (odd or < 2 nsteps, non-finite dt, repeats < 0),
 * DG_ESTATE (no workspace; no graph; build while dg_timing is active),
 * DG_EHIP (capture or instantiation refused by the runtime).              */
dg_status dg_rk_graph_build(dg_ctx* ctx, double dt, int nsteps);
dg_status dg_rk_graph_launch(dg_ctx* ctx, int repeats);

/* Ubar = (dL/dU (U))^T lam: vector-Jacobian product of dg_eval_rhs, i.e. the
 * transpose of the linearised split-form DG operator of paper Sec. 2.2 (BR1
 * lifting, two-point volume flux differencing, surface fluxes, surface
 * lifting and Jacobian scaling, each differentiated by hand).  U, lam and
 * Ubar are device arrays of 5 n_dof doubles in the state layout, caller
 * owned; Ubar must not overlap U or lam.  Needs a
 * workspace bound with_adjoint.  FP64 arithmetic.  The VJP calls cover
 * axis-aligned elements with isothermal or periodic ends (either flux pair,
 * either viscosity law); curved elements and the wall model get
 * DG_EUNSUPPORTED.  Non-smooth points (|.|, max, the entropy correction's
 * branch) take the derivative of the branch the values select.              */
dg_status dg_eval_rhs_vjp(dg_ctx* ctx, const double* U_dev, const double* lam_dev,
                          double* Ubar_dev, double t);

/* One RK step backwards: given U_n and lamU_np1 = dJ/dU_{n+1}, write
 * lamU_n = dJ/dU_n, the transpose of one step of the five-stage low-storage
 * RK scheme (paper Sec. 4) linearised at U_n: per stage in reverse order
 * lamG += B_s lamU, lamU += dt (dL/dU(U_{n,s}))^T lamG, lamG <- A_s lamG
 * (recomputes the five stage states internally in the context's precision;
 * the VJPs are FP64).  Device arrays of 5 n_dof doubles, caller owned;
 * lamU_n may alias lamU_np1.  Errors: DG_EINVAL, DG_ESTATE (no adjoint
 * workspace), DG_EUNSUPPORTED (curved elements, wall model).                */
dg_status dg_rk_step_vjp(dg_ctx* ctx, const double* U_n_dev, double t, double dt,
                         const double* lamU_np1_dev, double* lamU_n_dev);

/* Segment recompute for the checkpointed adjoint (the paper's RK scheme,
 * Sec. 4, run forward from a checkpoint): starting from U0, advance nsteps
 * steps of size dt and write the five stage input states U_{n,s} (s = 0..4;
 * U_{n,0} = U_n) of every step to the caller-owned device buffer stages, step
 * major: U_{n,s} starts at stages + (5 n + s) 5 n_dof; the buffer holds
 * 25 nsteps n_dof doubles and must not overlap U0.  The arithmetic is that of
 * dg_rk_step (the context's precision); afterwards the context's state is
 * U_nsteps and its RK register is overwritten.  Errors: DG_EINVAL (null
 * pointers, nsteps < 1, non-finite dt, U0 inside stages), DG_ESTATE (no
 * workspace).                                                                */
dg_status dg_rk_record_stages(dg_ctx* ctx, const double* U0_dev, double t, double dt, int nsteps,
                              double* stages_dev);

/* dg_rk_step_vjp with the step's five stage states read from stages_dev (the
 * 25 n_dof doubles dg_rk_record_stages wrote for that step) instead of
 * recomputed: lamU_n = dJ/dU_n from lamU_np1.  Needs a workspace bound
 * with_adjoint; FP64 arithmetic.                                             */
dg_status dg_rk_step_vjp_stages(dg_ctx* ctx, const double* stages_dev, double t, double dt,
                                const double* lamU_np1_dev, double* lamU_n_dev);

/* Wall faces of the mesh: 2 nb nc for every direction whose ends are walls
 * (nb, nc the element counts of the other two directions).  Host only.      */
dg_status dg_wall_faces(const dg_ctx* ctx, long long* n_faces);

/* Algebraic equilibrium wall-stress model (paper Sec. 3, one GPU lane per
 * wall-face node): at each node of each wall face, the state at the LGL node
 * n_wm (1..N, counted from the wall) of the wall-normal line through it, a
 * distance h_wm = (xi_nwm + 1) width / 2 from the wall; the wall-parallel
 * velocity u_par (normal component removed) and its direction t; the Van
 * Driest transform for an adiabatic wall, u_VD = a asin(u_par / a),
 * a^2 = 2 c_p T_w / r, T_w = T + r u_par^2 / (2 c_p), r = Pr^(1/3); wall
 * density p / (R T_w) and viscosity mu(T_w); u_tau from Spalding's law
 * h u_tau / nu_w = f(u_VD / u_tau), f(u+) = u+ + 0.1108 (exp(0.4 u+) - 1 -
 * 0.4 u+ - (0.4 u+)^2/2 - (0.4 u+)^3/6 - (0.4 u+)^4/24) (Newton, from below).
 * Writes tau_dev[(face 3 + c) (N+1)^2 + a + (N+1) b] = rho_w u_tau^2 t_c for
 * the dg_wall_faces faces in order: wall directions x, y, z; lower then upper
 * wall; wall elements with the first remaining element index fastest; face
 * nodes (a, b) = (j, k), (i, k), (i, j) for walls normal to x, y, z.
 * Errors: DG_EINVAL (null pointers, n_wm outside 1..N), DG_ESTATE (no
 * workspace).  Zero faces (no walls) is a no-op.                            */
dg_status dg_wall_stress(dg_ctx* ctx, const double* U_dev, int n_wm, double* tau_dev);

/* Volume-averaged kinetic energy J(U) = sum wJ |m|^2/(2 rho) / sum wJ with LGL
 * quadrature, written to J_dev[0] (device double).                           */
dg_status dg_kinetic_energy(dg_ctx* ctx, const double* U_dev, double* J_dev);

/* dJ/dU of dg_kinetic_energy (Euclidean gradient w.r.t. nodal values). */
dg_status dg_kinetic_energy_grad(dg_ctx* ctx, const double* U_dev, double* lam_dev);

/* STREAM triad a[i] = b[i] + s c[i] over n doubles on hip_stream (device
 * pointers, caller owned): the measured HBM ceiling the operator's achieved
 * bandwidth is compared with (24 bytes per element).  With 16-byte aligned
 * pointers every lane moves 16-byte pairs; otherwise 8-byte elements.
 * Asynchronous; no context needed.  Errors: DG_EINVAL (null pointer, n < 0),
 * DG_EHIP (launch failed).                                                   */
dg_status dg_stream_triad(const double* b_dev, const double* c_dev, double s, double* a_dev,
                          long long n, void* hip_stream);

/* Kernel timing for measurement.  dg_timing_begin(ctx, max_launches) makes the
 * following forward launches of the context record a HIP event on its stream
 * after each kernel (up to max_launches kernels; events are created here).
 * dg_timing_end waits for the stream and returns, per kernel class, the summed
 * device time in milliseconds and the launch count: [0] lifting, [1] right-hand
 * side / fused RK stage.  Errors: DG_EINVAL (bad arguments), DG_ESTATE (end
 * without begin), DG_EHIP.                                                   */
dg_status dg_timing_begin(dg_ctx* ctx, int max_launches);
dg_status dg_timing_end(dg_ctx* ctx, double ms[2], int count[2]);

/* Wait for the stream; report and clear the device status word. */
dg_status dg_sync(dg_ctx* ctx);

/* Text of the last error of this context (static per context). */
const char* dg_last_error(const dg_ctx* ctx);

/* Release the context (the workspace stays owned by the caller). */
dg_status dg_free(dg_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* DGSEM_H */
