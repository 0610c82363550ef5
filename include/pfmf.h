/*
 * pfmf: matrix-free coupled displacement / phase-field operator for MI355X.
 *
 * C ABI of the HIP library libpfmf.so. Every apply acts on a structured box of
 * order-p tensor-product hexahedra and computes, for the solution
 * z = [u_x, u_y, u_z, phi], the matrix-free residual
 *     R(z) = sum_e E_e^T [B_I; B_xi]^T W Lambda [f0; f1]
 * (Section 4, eq:matrix-free-residual-compact), its Jacobian action
 * (eq:matrix-free-jacobian) and its transpose. The pointwise integrands are the
 * Hencky / Peric-Dettmer block in series with the phase-field fracture element:
 *     f1 = [tau_degr F^-T ; s_phi (2 Gc l0 / c0) grad_X phi],  f0 = [0 ; s_phi L]
 * (eq:physical-residual-integrands with eq:mechanical-gradient-transformation and
 * eq:phase-gradient-transformation), with tau_degr from Box 1 / Box 2 degraded as
 * in eq:degraded-trial-stress and eq:linear-degraded-stress, and
 * L = g'(phi) H + Gc alpha'(phi) / (c0 l0) + zeta (phi - phi_n) / dt (eq:L-viscous).
 *
 * Conventions
 *  - Mesh: nx*ny*nz elements of order p (1..4) on [0,lx]x[0,ly]x[0,lz] (mm).
 *    Nodes are the Gauss-Lobatto-Legendre points of each element, numbered
 *    lexicographically x-fastest over (p*nx+1)(p*ny+1)(p*nz+1) lattice points.
 *    Quadrature is tensor Gauss-Legendre with Q = p+1 points per direction.
 *  - Nodal vectors are SoA [4][n_nodes] (u_x, u_y, u_z, phi).
 *  - Quadrature points are element-major (e = ex + nx*(ey + ny*ez)) and
 *    x-fastest inside the element: qp = e*Q^3 + qx + Q*(qy + Q*qz).
 *  - Per-point state is SoA [8][n_q] double: D (Voigt xx,yy,zz,yz,xz,xy) with
 *    D = Cin^-1_n - I (eq:inelasticity-be-update), the accumulated plastic strain
 *    and the history field H_n. Phase ids are uint8[n_q].
 *  - Units mm, MPa, s, N/mm.
 *
 * Memory and streams
 *  - All vector arguments of the apply calls are DEVICE pointers owned by the
 *    caller; the library never frees them. setup_mesh keeps the state, phase and
 *    phi_n pointers: they must stay valid (and unchanged unless re-linearised)
 *    for the lifetime of the context.
 *  - Applies are asynchronous on the given stream (a hipStream_t passed as
 *    void*, NULL = the legacy default stream) and never synchronise the host,
 *    except where stated.
 *  - The context owns only internal buffers (FP32 mirrors and the linearisation
 *    record, multigrid vectors, reduction scratch, the device error word). It is
 *    bound to the device current at setup; calls from another device fail with
 *    PF_EINVAL. Concurrent calls on one context from several host threads or
 *    streams are not supported (internal buffers are shared).
 *
 * Errors
 *  - Every call returns a pf_status. Negative values are errors; a message is
 *    available from pf_last_error() (thread-local). No C++ exception crosses the
 *    ABI. Output vectors must not alias inputs (PF_EINVAL).
 *  - A non-physical point (det F <= 0 or an eigenvalue of b_tr <= 0) makes the
 *    apply write non-finite values at the affected nodes and raise a sticky
 *    device flag; pf_check() synchronises the context's last stream and returns
 *    PF_ENONPHYSICAL once (then clears the flag).
 */
#ifndef PFMF_H
#define PFMF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PF_OK = 0,
  PF_EINVAL = -1,        /* bad argument (null, size, aliasing, wrong device) */
  PF_EHIP = -2,          /* a HIP runtime call failed */
  PF_ENOMEM = -3,        /* device allocation failed */
  PF_EUNSUPPORTED = -4,  /* order / configuration not built */
  PF_ENONPHYSICAL = -5,  /* a quadrature point left the physical domain */
  PF_ENOCONV = -6        /* an iterative solve missed its tolerance (the result is still written) */
} pf_status;

/* Structured box of order-p hexahedra (p = 1..4). */
typedef struct { int p; int nx, ny, nz; double lx, ly, lz; } pf_mesh_desc;

/* Material of one phase: Hencky Hooke branch (E [MPa], nu) plus, when plastic != 0,
 * one Prandtl branch (Box 2) with the hardening law eq:plasticity-strain-hardening-law,
 * sigma_y = sigma0 + H ebar_p + (sigma_inf - sigma0)(1 - exp(-voce_beta ebar_p))
 * (sigma0, H, sigma_inf [MPa]; voce_beta = 0 is linear hardening, else sigma_inf >=
 * sigma0 is required), and an overstress factor (1 + visc dgamma / dt) on the yield
 * stress (visc [s]; visc = 0 is Box 2 exactly). Linear hardening takes the closed-form
 * root of the consistency equation, Voce hardening Box 2's Newton iteration. Gc [N/mm]
 * is the critical energy release rate of the fracture element. */
typedef struct {
  double E, nu, Gc, sigma0, H, visc;
  int plastic;
  double sigma_inf, voce_beta;
} pf_phase;

/* Extra rheological branch in parallel with a phase's block (Section 2.3 and Box 1:
 * tau = sum_k tau_k, psi = sum_k psi_k, each branch with its own Cin^-1): kind
 * PF_BRANCH_HOOKE (spring E [MPa], nu; Cin^-1 = I), PF_BRANCH_MAXWELL (spring plus the
 * deviatoric viscosity eta_d [MPa s]; closed-form update
 * eq:viscoelasticity-deviatoric-strain-update-hencky with the degraded modulus g mu,
 * eq:principal-directions-format-1) or PF_BRANCH_PRANDTL (spring plus sigma0, H, visc,
 * sigma_inf, voce_beta as in pf_phase); PF_BRANCH_NONE leaves the slot empty. Every
 * branch is degraded by the Amor split of its own trial volumetric strain; the point's
 * psi^+ (history field and phase-field residual) is the sum over the block and the
 * branches. */
#define PF_BRANCH_NONE 0
#define PF_BRANCH_HOOKE 1
#define PF_BRANCH_MAXWELL 2
#define PF_BRANCH_PRANDTL 3
#define PF_MAX_EXTRA_BRANCHES 2
typedef struct {
  int kind;
  double E, nu, eta_d, sigma0, H, visc, sigma_inf, voce_beta;
} pf_branch;

/* Fracture element and time step: length scale l0 [mm], residual stiffness eta
 * (eq:degr-funct), damage viscosity zeta [MPa s] (Section 3.1), time step dt [s],
 * global phase-field residual scale s_phi (eq:damage-residual-scaling), AT model
 * 1 or 2 (eq:AT1-AT2). */
typedef struct { double l0, eta, zeta, dt, s_phi; int at; } pf_fracture;

/* p-multigrid V-cycle options. Levels as set by pf_set_pmg_levels (default p, p-1,
 * ..., 1), all evaluated at the fine quadrature; coarse_p must equal the last order. cheb_degree smoothing steps of Chebyshev with
 * point-Jacobi before and after the coarse correction; coarse_sweeps Chebyshev
 * applications on the coarsest level. Zero fields take defaults (3, 1, 4). */
typedef struct { int cheb_degree; int coarse_p; int coarse_sweeps; int reserved; } pf_pmg_opts;

typedef struct pf_ctx pf_ctx;

/* Create a context. qp_phase (uint8[n_q]), qp_state (double[8][n_q]) and phi_n
 * (double[n_nodes], the converged phase field of the previous step) are device
 * pointers kept by the context. n_phases in 1..255. stream: void* hipStream_t. */
pf_status pf_setup_mesh(const pf_mesh_desc* mesh, const pf_phase* phases, int n_phases,
                        const pf_fracture* fracture, const uint8_t* qp_phase,
                        const double* qp_state, const double* phi_n, void* stream,
                        pf_ctx** out);

/* Hexahedral mesh given by a table restriction (the general element restriction E and
 * P of Section 4's compact residual, eq:matrix-free-residual-compact, as on the paper's
 * unstructured meshes): n_elem elements of order p (2, 3 or 4) over n_nodes nodes. */
typedef struct { int p; int64_t n_elem, n_nodes; } pf_table_mesh_desc;

/* Create a context on a mesh given by its element-to-node table. conn: device
 * int32[n_elem][(p+1)^3], conn[e (p+1)^3 + a] = global node of local node
 * a = ax + (p+1)(ay + (p+1) az) of element e in the element's own reference coordinates
 * (any orientation, any node numbering); X: device double[3][n_nodes], node positions
 * (every element is mapped, Section 4's isoparametric map; X is read once, not kept).
 * Quadrature points stay element-major, qp = e (p+1)^3 + qx + (p+1)(qy + (p+1) qz) in
 * the element's reference coordinates; qp_phase, qp_state, phi_n and the nodal vectors are
 * as for pf_setup_mesh with n_nodes and n_q = n_elem (p+1)^3. conn is kept by the context
 * (valid and unchanged for its lifetime). The call reads the table once (host copy,
 * synchronising `stream`) to build the node-to-(element, local node) map of its
 * transpose, computes the geometry record (80 bytes per point) and allocates the element
 * vectors (n_elem x 4 (p+1)^3 doubles). The FP64 residual, Jacobian and adjoint then
 * gather through the table and scatter deterministically: each element vector is stored,
 * and every node sums its entries in element order (no atomics). The multigrid, the
 * Newton step, the state commit, extra branches, pf_set_geometry and
 * pf_apply_adjoint_noalloc need the box lattice and return PF_EUNSUPPORTED on such a
 * context. Errors: PF_EINVAL for a node id outside 0..n_nodes-1, an inverted element
 * (det J <= 0), a phase id >= n_phases or sizes beyond 32-bit indices;
 * PF_EUNSUPPORTED for p other than 2, 3, 4; PF_ENOMEM, PF_EHIP. */
pf_status pf_setup_mesh_table(const pf_table_mesh_desc* mesh, const int32_t* conn, const double* X,
                              const pf_phase* phases, int n_phases, const pf_fracture* fracture,
                              const uint8_t* qp_phase, const double* qp_state, const double* phi_n,
                              void* stream, pf_ctx** out);

/* Sizes of the fine level. Any output pointer may be NULL. */
pf_status pf_sizes(const pf_ctx* ctx, int64_t* n_nodes, int64_t* n_q, int64_t* n_dof);

/* Attach n_extra (0..PF_MAX_EXTRA_BRANCHES) extra branches to every phase:
 * branches[n_phases][n_extra] in host memory (copied), xstate a device pointer kept by
 * the context, double[7*n_extra][n_q]: rows 7j..7j+5 the D = Cin^-1 - I (Voigt) of
 * extra branch j, row 7j+6 its accumulated plastic strain (a Hooke branch reads none of
 * them). n_extra = 0 detaches (branches and xstate may then be NULL). Orders 2-4; the
 * FP64 residual, Jacobian and adjoint (with the block's parameter partials) include the
 * branches, and so does the linearisation: pf_linearize stores one record layer per
 * branch (the block's layer holds the switch and dL/dphi of the total psi^+), which the
 * FP32 levels, the V-cycle, pf_apply_jacobian_lin and pf_newton_step sum over; the
 * record grows to (1 + n_extra) layers. The call invalidates the linearisation and
 * synchronises the device before it frees the previous branch tables (applies still in
 * flight on any stream may read them), so it is not for use inside a stream capture.
 * The state commit with branches is pf_commit_state_branches.
 * Errors: PF_EINVAL for a bad kind or parameter (E > 0, -1 < nu < 0.5, eta_d > 0,
 * sigma0, H, visc, voce_beta >= 0, sigma_inf >= sigma0 with Voce), PF_EUNSUPPORTED at
 * p = 1, PF_ENOMEM / PF_EHIP from the device copy. */
pf_status pf_set_branches(pf_ctx* ctx, const pf_branch* branches, int n_extra, const double* xstate);

/* Mapped (curved) elements, the isoparametric map of Section 4: X is a device pointer to
 * double[3][n_nodes], the position of every node (rows x, y, z; node order as z). The call
 * computes, once, a per-point geometry record of 10 doubles (J^-1 and the weight times
 * det J, 80 bytes per point, owned by the context, plus an FP32 copy of 40 bytes per point
 * for the FP32 levels) from which the applies take their gradients and weights; X itself
 * is not kept. X = NULL returns to
 * the box. Orders 2-4. The call invalidates the linearisation, synchronises the device
 * before it frees the previous record (applies in flight may read it) and synchronises
 * the stream after building the new one. Everything else follows the geometry too: the state commit, the linearisation
 * (records, FP32 levels evaluated at the fine points with the fine J^-1, their Jacobi
 * diagonals, the order-1 element matrices), pf_apply_jacobian_lin, the V-cycle and
 * pf_newton_step.
 * Extra branches in parallel (pf_set_branches) combine with it.
 * Errors: PF_EINVAL when some point has det J <= 0 (the geometry stays detached),
 * PF_EUNSUPPORTED at p = 1, PF_ENOMEM, PF_EHIP. */
pf_status pf_set_geometry(pf_ctx* ctx, const double* X, void* stream);

/* Replace the per-phase parameters (Gc, sigma0, visc) from host memory
 * params[n_phases][3] (the material of the residual, Sections 2-3; the parameters the
 * adjoint differentiates). Stream-ordered and asynchronous: the tables are staged in
 * pinned host memory owned by the context and copied on `stream`, so applies enqueued
 * on that stream before the call use the old values and later ones the new; params may
 * be reused as soon as the call returns. The host waits only when four earlier uploads
 * are still queued. Values equal to the current ones upload nothing and keep the
 * linearisation; other values invalidate it. Errors: PF_EINVAL for a negative value,
 * sigma0 = 0 in a plastic phase or sigma0 above a Voce phase's sigma_inf. */
pf_status pf_set_params(pf_ctx* ctx, const double* params, void* stream);

/* r = R(z). z, r: device double[4][n_nodes]. */
pf_status pf_apply_residual(pf_ctx* ctx, const double* z, double* r, void* stream);

/* y = J(z) dz, the exact directional derivative of R at z (Appendices B-C),
 * recomputed from z and the state (nothing stored). z, dz, y: double[4][n_nodes]. */
pf_status pf_apply_jacobian(pf_ctx* ctx, const double* z, const double* dz, double* y,
                            void* stream);

/* gz = J(z)^T v and gparams[n_phases][3] = v^T dR/d(Gc, sigma0, visc) summed per phase
 * (device double). The pointwise linearisation is recomputed, not stored. */
pf_status pf_apply_adjoint(pf_ctx* ctx, const double* z, const double* v, double* gz,
                           double* gparams, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): pf_apply_adjoint with no allocation of
 * any kind. Same arguments, results and errors as pf_apply_adjoint (gz and gparams equal
 * to it up to the order of the final additions); the scatter-add takes the
 * eight colour launches, which write gz directly, and the per-brick (order 4:
 * per-element) parameter partials go to a static device array of PF_NOALLOC_PARTIALS
 * doubles (4 MiB) that each GPU the library runs on holds until the process ends. Every
 * call overwrites all partials it reads, so nothing carries over between calls; calls
 * that overlap on one GPU (several streams, threads or contexts at once) race on that
 * array and must be serialised by the caller. Errors: PF_EINVAL when
 * 3 n_phases x (number of 2x2x2-element bricks, or of elements at order 4) exceeds
 * PF_NOALLOC_PARTIALS, PF_EUNSUPPORTED on a table-restriction context, the errors of
 * pf_apply_adjoint otherwise. */
#define PF_NOALLOC_PARTIALS (1 << 19)
pf_status pf_apply_adjoint_noalloc(pf_ctx* ctx, const double* z, const double* v, double* gz,
                                   double* gparams, void* stream);

/* Linearise at z for the FP32 multigrid: the return-mapping, split and history
 * decisions, their scalars, the principal frame of b_tr (a unit quaternion, its three
 * smallest components), the principal trial log strains and the off-diagonal tangent
 * factors are taken in FP64 and stored per point (and per branch, see pf_set_branches)
 * as an FP32 record of 15 values and a
 * flag byte (Appendices A-C evaluated once), with an FP32 mirror of u; assembles an
 * order-1 level into a block stencil and the Galerkin stencils of any coarser order-1
 * lattices below it; builds every level's point-Jacobi
 * diagonal and Chebyshev bounds (power iteration on the device). Synchronises the
 * stream once. */
pf_status pf_linearize(pf_ctx* ctx, const double* z, void* stream);

/* Multigrid level orders, fine first: orders[0] = p > orders[1] > ... >= 1,
 * 2 <= n_levels <= 8 (n_levels = 0 restores the default p, p-1, ..., 1). Every level
 * is evaluated at the fine quadrature. After the first order 1 the list may repeat 1:
 * each further 1 is the order-1 lattice with half the elements per direction (the
 * element counts must be even), trilinear interpolation from it, and as its operator the
 * Galerkin product P^T A P of the level above, formed by pf_linearize as a block stencil
 * (a geometric coarse hierarchy below the p-levels, e.g. 4, 2, 1, 1, 1). PF_EINVAL for
 * other lists or a lattice that cannot be halved. Frees the hierarchy: call pf_linearize
 * again. */
pf_status pf_set_pmg_levels(pf_ctx* ctx, const int* orders, int n_levels);

/* Context options (pf_set_option).
 * PF_OPT_SCATTER: how the FP64 residual, Jacobian and adjoint and the record applies
 * (FP32 levels, stored FP64 Jacobian) on order-2, 3 and 4 meshes add the element
 * contributions into their output (the scatter-add E^T P^T of Section 4).
 * 1 = eight colour launches by brick (order 4: element) parity that write the output
 * directly; 2 = the elements' sums stored in a context-owned buffer (allocated on first
 * use; orders 2, 3: per 2x2x2-element brick, 4 x (2p+1)^3 values; order 4: per element,
 * 4 x 125 values; FP64 and FP32 separately), then a node gather that adds them in a
 * fixed order; 0 = automatic (default): 2 while the FP64 buffer stays within
 * PF_SCATTER_AUTO_BYTES, else 1. Both are deterministic and differ only in the order of
 * the final additions. Order-1 meshes ignore the option (8 colours). */
#define PF_OPT_SCATTER 1
#define PF_SCATTER_AUTO_BYTES (4LL << 30)
/* PF_OPT_STORE_LIN64 (default 1): pf_linearize also stores the linearisation record
 * in FP64 (15 doubles per point, sharing the FP32 record's flag bytes) and a copy of u,
 * for pf_apply_jacobian_lin; 0 skips both. */
#define PF_OPT_STORE_LIN64 2
pf_status pf_set_option(pf_ctx* ctx, int option, int value);

/* Dirichlet faces for the multigrid and the Newton step: bit f of face_fields[k]
 * constrains field f (u_x, u_y, u_z, phi) on face k (x = 0, x = lx, y = 0, y = ly,
 * z = 0, z = lz) (the essential conditions of the weak form, Section 3). With faces set,
 * the FP32 level operators return M A x (M zeroes constrained entries), the V-cycle
 * works on the masked right-hand side, and its output vanishes on constrained
 * entries. The FP64 applies are unaffected. Call pf_linearize again afterwards. */
pf_status pf_set_dirichlet(pf_ctx* ctx, const uint32_t face_fields[6]);

/* State commit after a converged step (Section 2, exponential-map update): from the
 * converged z and the context's state, state_out[8][n_q] (device double, same layout)
 * gets D_{n+1} = F^-1 b^e F^-T - I with b^e = exp(2 eps^e), eps^e the trial log strain
 * with its deviator scaled by the return factor, ebar_p + dgamma and max(H_n, psi^+).
 * state_out must not alias the context's state or z. To advance a step, copy it into
 * the state buffer given to pf_setup_mesh (and phi into phi_n) once the stream is done. */
pf_status pf_commit_state(pf_ctx* ctx, const double* z, double* state_out, void* stream);

/* The same with extra branches attached (Box 1 step 4 for every branch): state_out as
 * above, with the history field of the point's total psi^+; xstate_out (device double,
 * the layout of the xstate given to pf_set_branches) gets each Maxwell or Prandtl branch's
 * D_{n+1} by the same exponential map with its own return factor and its ebar_p + dgamma;
 * the rows of Hooke branches and empty slots are copied. xstate_out must not alias the
 * context's states, state_out or z. pf_commit_state returns PF_EUNSUPPORTED while
 * branches are attached, this call PF_EINVAL while none is. */
pf_status pf_commit_state_branches(pf_ctx* ctx, const double* z, double* state_out, double* xstate_out,
                                   void* stream);

/* Newton step options: relative tolerance of the linear solve (default 1e-8),
 * FGMRES restart length (30, at most 60), iteration limit (300), the V-cycle
 * smoother (Chebyshev degree 3, 32 coarsest sweeps), and the Krylov method:
 * PF_KRYLOV_FGMRES (0, default; the GMRES of Section 5 with the V-cycle as flexible
 * right preconditioner) or PF_KRYLOV_CG (1; preconditioned conjugate gradients with
 * the same V-cycle, which assume a symmetric positive definite system: the coupled
 * Jacobian is not one in general, so CG stops at the first breakdown, p^T J p <= 0
 * or r^T M r <= 0, and reports it). Zero fields take defaults. */
#define PF_KRYLOV_FGMRES 0
#define PF_KRYLOV_CG 1
typedef struct {
  double rtol;
  int restart, max_iters, cheb_degree, coarse_sweeps;
  int krylov;
  int reserved[2];
} pf_newton_opts;

/* Newton step report: Krylov iterations, convergence flag, ||b|| with b = -M R(z),
 * the solver's residual (FGMRES estimate, CG recurrence), the true residual
 * ||b - M J dz||, host wall times (linearisation, whole step) in milliseconds, the
 * number of FGMRES iterations whose Gram-Schmidt needed the second (refinement) pass,
 * the Krylov method used, and whether CG broke down. */
typedef struct {
  int iterations, converged;
  double res0, res_lin, res_true;
  double t_linearize_ms, t_total_ms;
  int refinements;
  int krylov, breakdown;
} pf_newton_stats;

/* One Newton update z += dz of the coupled problem with the Dirichlet faces of
 * pf_set_dirichlet: M J(z) dz = -M R(z) (M zeroes constrained entries, which z must
 * already hold at their prescribed values), solved by restarted flexible GMRES with
 * the FP64 Jacobian apply (from the stored FP64 linearisation when PF_OPT_STORE_LIN64
 * is on, p >= 2 and no extra branch is attached, else recomputed; the reported true
 * residual always uses the recomputed one) and one FP32 p-multigrid V-cycle per
 * iteration as right
 * preconditioner (re-linearised at z; the paper's solver is GMRES with p-multigrid,
 * Section 5). Allocates its Krylov workspace ((2 restart + 4) vectors of 4 n_nodes
 * doubles) on first use and keeps it. Synchronises the stream. Returns PF_ENOCONV when
 * the tolerance is missed (z is still updated). */
pf_status pf_newton_step(pf_ctx* ctx, double* z, const pf_newton_opts* opts, pf_newton_stats* stats,
                         void* stream);

/* Number of multigrid levels available after pf_linearize (level 0 = fine), and the
 * order and node count of one level. */
pf_status pf_level_info(const pf_ctx* ctx, int level, int* p, int64_t* n_nodes);

/* y = J dz in FP32 on one level (level 0 = fine order p; the orders as set by
 * pf_set_pmg_levels, default p - l), evaluated at the fine quadrature with the record of
 * the last pf_linearize (a coarser order-1 lattice: its Galerkin stencil).
 * dz, y: device float[4][n_nodes(level)]. */
pf_status pf_apply_jacobian_f32(pf_ctx* ctx, int level, const float* dz, float* y,
                                void* stream);

/* FP64 Jacobian action at the last linearisation point z (Section 4, with the pointwise
 * linearisation of Appendices A-C evaluated once by pf_linearize and stored): y = J(z) dz
 * from the stored FP64 record and the copy of u, orders 2-4. Same operator as
 * pf_apply_jacobian at that z (the decisions, frame and coefficients are the FP64 ones;
 * the results differ by rounding only), without recomputing the eigen-frame and return
 * mapping at every apply: for Krylov iterations at one Newton iterate. dz, y: device
 * [4][n_nodes] FP64; y must not alias dz. Needs pf_linearize with PF_OPT_STORE_LIN64 on
 * (PF_EINVAL otherwise); pf_set_params invalidates the linearisation. */
pf_status pf_apply_jacobian_lin(pf_ctx* ctx, const double* dz, double* y, void* stream);

/* Level transfer: prolongation xf = P xc (coarse level l+1 -> level l, exact
 * interpolation of the coarse field at the fine nodes; trilinear between order-1
 * lattices) and restriction rc = P^T rf. Device float[4][n_nodes(level)]. */
pf_status pf_prolong(pf_ctx* ctx, int level, const float* xc, float* xf, void* stream);
pf_status pf_restrict(pf_ctx* ctx, int level, const float* rf, float* rc, void* stream);

/* Point-Jacobi diagonal of one level (float[4][n_nodes(level)], device). */
pf_status pf_level_diagonal(pf_ctx* ctx, int level, float* diag, void* stream);

/* One FP32 p-multigrid V-cycle for J x = b at the last linearisation, starting
 * from x = 0. b, x: device float[4][n_nodes] on the fine level. */
pf_status pf_pmg_vcycle(pf_ctx* ctx, const float* b, float* x, const pf_pmg_opts* opts,
                        void* stream);

/* Synchronise and report the sticky non-physical flag (PF_ENONPHYSICAL once). */
pf_status pf_check(pf_ctx* ctx);

/* Free the context and its internal buffers (synchronises its streams). */
void pf_destroy(pf_ctx* ctx);

/* Last error message of the calling thread ("" if none). */
const char* pf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
