/*
 * CPU oracle for the coupled displacement / phase-field operator.
 *
 * TEST INFRASTRUCTURE ONLY. This is a plain, slow FP64 reference used by the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark. The
 * product path (the HIP library) never links, loads or calls it, and it shares
 * no code, header or table with that library.
 *
 * Method: finite-strain Hencky material with a Peric-Dettmer inelastic block
 * (Hooke branch, or one Prandtl branch with linear or Voce hardening and an
 * overstress factor, optionally with up to two extra Hooke / Maxwell / Prandtl
 * branches in parallel) in series with a phase-field fracture element (Sections 2-3 of the
 * paper), discretised with tensor-product hexahedra and Gauss quadrature
 * (Section 4). Element operators use dense element matrices built from the 1-D
 * Lagrange basis (no sum factorisation).
 *
 * Pins (tests/test_oracle_pins.py, tests/test_oracle_commit_pins.py,
 * tests/test_oracle_branch_pins.py) tie every function here to closed forms,
 * library routines, invariants or finite differences. Parity unpinned: the overstress factor (1 + visc dgamma / dt) of the
 * Prandtl branch is a reading, not the paper's; it is pinned only at visc = 0
 * (Box 2), by its own root-finding (bisection, Newton) and by finite differences.
 * The global phase-field scale s_phi is an input, not derived here.
 *
 * Conventions (shared interface, see inputs.py): nodes lexicographic x-fastest,
 * z = SoA [4][n_nodes] (u_x,u_y,u_z,phi), qp = e*Q^3 + qx + Q*(qy + Q*qz),
 * state = SoA [8][n_q] (D xx,yy,zz,yz,xz,xy = Cin^-1 - I; ebar_p; H_n),
 * extra branches' state = SoA [7*n_extra][n_q] (D, ebar_p per branch),
 * phase = uint8[n_q]. Units mm, MPa, s, N/mm.
 */
#ifndef PF_ORACLE_H
#define PF_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* X: optional positions of the nodes [3][n_nodes] (an isoparametric map of every element,
 * Section 4); NULL = the box [0,lx]x[0,ly]x[0,lz] with affine elements.
 * conn: optional element restriction as a table (the general E and P of Section 4's
 * compact residual): conn[e*(p+1)^3 + a] is the global node of local node
 * a = ax + (p+1)(ay + (p+1) az) of element e, for e < n_elem, nodes < n_nodes; it needs X
 * (every element is mapped) and then replaces the lattice numbering (nx, ny, nz, lx, ly,
 * lz are ignored). NULL = the box lattice (n_elem, n_nodes ignored). */
typedef struct {
  int p, q, nx, ny, nz;
  double lx, ly, lz;
  const double* X;
  const int32_t* conn;
  int64_t n_elem, n_nodes;
} or_mesh;
/* sigma_inf, voce_beta: Voce term (sigma_inf - sigma0)(1 - exp(-voce_beta ebar_p)) of the
 * hardening law; voce_beta = 0 is linear hardening. */
typedef struct { double E, nu, Gc, sigma0, H, visc; int plastic; double sigma_inf, voce_beta; } or_phase;
typedef struct { double l0, eta, zeta, dt, s_phi; int at; } or_frac;

/* Extra rheological branch in parallel with a phase's block (Section 2.3, Box 1):
 * its own spring (E, nu); a Maxwell branch's deviatoric viscosity eta_d [MPa s]; a
 * Prandtl branch's hardening and overstress as in or_phase. Kind OR_BR_NONE skips
 * the slot. The extra state of branch j is 7 rows of [7*n_extra][n_q]: D[6] (Voigt,
 * Cin^-1 - I) and ebar_p; an extra Hooke branch reads none. */
enum { OR_BR_NONE = 0, OR_BR_HOOKE = 1, OR_BR_MAXWELL = 2, OR_BR_PRANDTL = 3 };
#define OR_MAX_EXTRA 2
typedef struct {
  int kind;
  double E, nu, eta_d, sigma0, H, visc, sigma_inf, voce_beta;
} or_branch;

/* Every pointwise quantity the tests look at. */
typedef struct {
  double P[9];        /* first Piola stress P = tau_degr F^-T, row-major P[i*3+J] */
  double f0;          /* s_phi * L */
  double f1[3];       /* s_phi * (2 Gc l0 / c0) * grad_X phi */
  double tau[6];      /* degraded Kirchhoff stress, Voigt xx,yy,zz,yz,xz,xy */
  double beta[3];     /* eigenvalues of b_tr - I, ascending */
  double eps[3];      /* principal trial log strains */
  double theta;       /* trace of the log strain */
  double q;           /* undegraded trial von Mises stress */
  double dgamma;      /* plastic multiplier increment */
  double c;           /* radial-return factor on the deviatoric strain */
  double psi_plus;    /* tensile energy psi^+ */
  double H;           /* max(H_n, psi^+) */
  double L;           /* local phase-field residual */
  double g;           /* degradation g(phi) */
  int plastic_active; /* 1 if the (degraded) yield check failed */
  int nonphysical;    /* 1 if 1+beta_i <= 0 or det F <= 0 */
} or_qp_out;

/* 1-D rules. Gauss-Legendre points/weights and GLL points on [-1,1]. */
void or_gauss(int n, double* x, double* w);
void or_gll(int n, double* x);

/* Pointwise residual integrand (steps R1-R12). G = grad_X u row-major. */
void or_qf_residual(const or_phase* ph, const or_frac* fr, const double G[9],
                    double phi, const double gphi[3], double phi_n,
                    const double st[8], or_qp_out* out);

/* Pointwise directional derivative (steps J1-J12): (dG, dphi, dgphi) -> (dP, df0, df1). */
void or_qf_jacobian(const or_phase* ph, const or_frac* fr, const double G[9],
                    double phi, const double gphi[3], double phi_n,
                    const double st[8], const double dG[9], double dphi,
                    const double dgphi[3], double dP[9], double* df0, double df1[3]);

/* The same with n_extra extra branches xb[n_extra] in parallel (total stress and
 * psi^+ summed over the branches; xs = the extra states, 7 values per branch). */
void or_qf_residual_mb(const or_phase* ph, const or_branch* xb, int n_extra, const or_frac* fr,
                       const double G[9], double phi, const double gphi[3], double phi_n,
                       const double st[8], const double* xs, or_qp_out* out);
void or_qf_jacobian_mb(const or_phase* ph, const or_branch* xb, int n_extra, const or_frac* fr,
                       const double G[9], double phi, const double gphi[3], double phi_n,
                       const double st[8], const double* xs, const double dG[9], double dphi,
                       const double dgphi[3], double dP[9], double* df0, double df1[3]);

/* Pointwise partial derivatives of (P, f0, f1) with respect to the phase's
 * (Gc, sigma0, visc): dP[k*9+..], df0[k], df1[k*3+..] for k = 0,1,2. */
void or_qf_param_partials(const or_phase* ph, const or_frac* fr, const double G[9],
                          double phi, const double gphi[3], double phi_n,
                          const double st[8], double dP[27], double df0[3], double df1[9]);

/* Global applies. elems = list of element ids to include (NULL = all).
 * xbr[nph][n_extra] extra branches per phase (n_extra = 0..OR_MAX_EXTRA; NULL with 0),
 * xstate = their states [7*n_extra][n_q] (NULL with 0).
 * Output vectors are zeroed first and hold the sum over the listed elements.
 * Return 0 on success, 1 if any quadrature point was non-physical, -1 on bad args. */
int or_residual(const or_mesh* m, const or_phase* ph, int nph, const or_branch* xbr, int n_extra,
                const or_frac* fr, const uint8_t* phase, const double* state, const double* xstate,
                const double* phi_n, const double* z, double* r, const int32_t* elems, int64_t n_elems);
int or_jacobian(const or_mesh* m, const or_phase* ph, int nph, const or_branch* xbr, int n_extra,
                const or_frac* fr, const uint8_t* phase, const double* state, const double* xstate,
                const double* phi_n, const double* z, const double* dz, double* y,
                const int32_t* elems, int64_t n_elems);
/* gz = J^T v (built from the explicit transpose of each point's tangent matrix);
 * gparams[nph*3] = v^T dR/d(Gc, sigma0, visc) summed per phase. */
int or_adjoint(const or_mesh* m, const or_phase* ph, int nph, const or_branch* xbr, int n_extra,
               const or_frac* fr, const uint8_t* phase, const double* state, const double* xstate,
               const double* phi_n, const double* z, const double* v, double* gz, double* gparams,
               const int32_t* elems, int64_t n_elems);

/* Dense element Jacobian (4*P^3 x 4*P^3, row-major, dof = field*P^3 + local node)
 * of element e. */
int or_element_jacobian(const or_mesh* m, const or_phase* ph, int nph, const or_branch* xbr,
                        int n_extra, const or_frac* fr, const uint8_t* phase, const double* state,
                        const double* xstate, const double* phi_n, const double* z, int64_t e,
                        double* Ke);

/* State commit after a converged step: new per-point state (D, ebar_p, H) from the
 * converged fields (exponential-map update of Section 2, history maximum of Section 3). */
void or_qf_commit(const or_phase* ph, const or_frac* fr, const double G[9], double phi,
                  const double st[8], double st_new[8]);
int or_commit_state(const or_mesh* m, const or_phase* ph, int nph, const or_frac* fr,
                    const uint8_t* phase, const double* state, const double* z, double* state_new);
/* With extra branches (Box 1 step 4 for every branch): the block's history field takes the
 * point's total psi^+; each Maxwell or Prandtl branch gets its own exponential-map update
 * and ebar_p + dgamma in xs_new / xstate_new; Hooke rows and empty slots are copied. */
void or_qf_commit_mb(const or_phase* ph, const or_branch* xb, int n_extra, const or_frac* fr,
                     const double G[9], double phi, const double st[8], const double* xs, double st_new[8],
                     double* xs_new);
int or_commit_state_mb(const or_mesh* m, const or_phase* ph, int nph, const or_branch* xbr, int n_extra,
                       const or_frac* fr, const uint8_t* phase, const double* state, const double* xstate,
                       const double* z, double* state_new, double* xstate_new);

/* Number of OpenMP threads the applies use (1 when built without OpenMP). */
/* (ln b_i - ln b_j) / (b_i - b_j) for b = 1 + beta (the off-diagonal factor of the
 * principal-direction tangent, Appendix B), finite as b_i -> b_j. */
double or_log_divdiff(double bi_m1, double bj_m1);
int or_num_threads(void);
void or_set_num_threads(int n);  /* OpenMP threads of the element loops (timing only) */

#ifdef __cplusplus
}
#endif
#endif
