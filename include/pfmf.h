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
  PF_ENONPHYSICAL = -5   /* a quadrature point left the physical domain */
} pf_status;

/* Structured box of order-p hexahedra (p = 1..4). */
typedef struct { int p; int nx, ny, nz; double lx, ly, lz; } pf_mesh_desc;

/* Material of one phase: Hencky Hooke branch (E [MPa], nu) plus, when plastic != 0,
 * one Prandtl branch (Box 2) with initial yield sigma0 [MPa], linear hardening H [MPa]
 * (eq:plasticity-strain-hardening-law without the Voce term) and an overstress factor
 * (1 + visc dgamma / dt) on the yield stress (visc [s]; visc = 0 is Box 2 exactly).
 * Gc [N/mm] is the critical energy release rate of the fracture element. */
typedef struct { double E, nu, Gc, sigma0, H, visc; int plastic; } pf_phase;

/* Fracture element and time step: length scale l0 [mm], residual stiffness eta
 * (eq:degr-funct), damage viscosity zeta [MPa s] (Section 3.1), time step dt [s],
 * global phase-field residual scale s_phi (eq:damage-residual-scaling), AT model
 * 1 or 2 (eq:AT1-AT2). */
typedef struct { double l0, eta, zeta, dt, s_phi; int at; } pf_fracture;

/* p-multigrid V-cycle options. Levels p, p-1, ... down to coarse_p (>= 1), all
 * evaluated at the fine quadrature. cheb_degree smoothing steps of Chebyshev with
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

/* Sizes of the fine level. Any output pointer may be NULL. */
pf_status pf_sizes(const pf_ctx* ctx, int64_t* n_nodes, int64_t* n_q, int64_t* n_dof);

/* Replace the per-phase parameters (Gc, sigma0, visc) from host memory
 * params[n_phases][3]. Takes effect for applies enqueued after the call. */
pf_status pf_set_params(pf_ctx* ctx, const double* params);

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

/* Linearise at z for the FP32 multigrid: the return-mapping, split and history
 * decisions and their scalars are taken in FP64 and stored per point as an FP32
 * record together with FP32 mirrors of z and D; builds every level's point-Jacobi
 * diagonal and Chebyshev bounds. Synchronises the stream (eigenvalue estimates). */
pf_status pf_linearize(pf_ctx* ctx, const double* z, void* stream);

/* Number of multigrid levels available after pf_linearize (level 0 = fine), and the
 * order and node count of one level. */
pf_status pf_level_info(const pf_ctx* ctx, int level, int* p, int64_t* n_nodes);

/* y = J dz in FP32 on one level (level 0 = fine order p; level l has order p-l),
 * evaluated at the fine quadrature with the record of the last pf_linearize.
 * dz, y: device float[4][n_nodes(level)]. */
pf_status pf_apply_jacobian_f32(pf_ctx* ctx, int level, const float* dz, float* y,
                                void* stream);

/* Level transfer: prolongation xf = P xc (coarse level l+1 -> level l, exact
 * interpolation of the coarse field at the fine nodes) and restriction rc = P^T rf.
 * Device float[4][n_nodes(level)]. */
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
