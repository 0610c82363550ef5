// Host side shared by the library's translation units: the context, error reporting,
// and the declarations of the FP64 operator dispatch (one translation unit per apply
// mode instantiates it, so that the kernels compile in parallel).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "pfmf.h"
#include "pf_ops.hpp"
#include "pf_mg.hpp"
#include "pf_step.hpp"

// Sets the calling thread's last-error message and returns s.
pf_status fail(pf_status s, const char* fmt, ...);

#define HIPCHK(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess) return fail(PF_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

using pfmf::DevTables;
using pfmf::DevTablesF;
using pfmf::DirMask;
using pfmf::FracParams;
using pfmf::MatParams;
using pfmf::MGState;
using pfmf::XBranch;

struct pf_ctx {
  int device = 0;
  pf_mesh_desc mesh{};
  int P = 0, Q = 0;
  int nx1 = 0, ny1 = 0, nz1 = 0;
  int64_t n_nodes = 0, n_q = 0;
  int nbx = 0, nby = 0, nbz = 0, n_bricks = 0;
  int n_parts = 0;  // slots of the adjoint's parameter partials
  bool has_voce = false;  // some plastic phase hardens by the Voce law
  int colour_base[9] = {0};
  std::vector<pf_phase> phases;
  pf_fracture fr{};
  const uint8_t* qp_phase = nullptr;
  const double* qp_state = nullptr;
  const double* phi_n = nullptr;
  // extra branches in parallel (pf_set_branches)
  int n_extra = 0;
  bool xvoce = false;  // some extra Prandtl branch hardens by the Voce law
  XBranch* d_xb = nullptr;
  MatParams<double>* d_xmats64 = nullptr;  // the same branches' materials for the record applies
  MatParams<float>* d_xmatsf = nullptr;
  const double* xstate = nullptr;
  // mapped elements (pf_set_geometry): per-point J^-1 and weights [10][n_q]
  double* d_qd = nullptr;
  float* d_qd32 = nullptr;  // the same record in FP32 for the FP32 levels
  // device buffers
  DevTables* d_tab = nullptr;
  DevTablesF* d_tabf = nullptr;
  MatParams<double>* d_mats = nullptr;
  MatParams<float>* d_matsf = nullptr;
  double* d_gpart = nullptr;
  double* d_ebuf = nullptr;  // brick-buffer scatter (allocated on first use)
  int scatter_mode = 0;      // PF_OPT_SCATTER
  bool store_lin64 = true;   // PF_OPT_STORE_LIN64
  // table restriction (pf_setup_mesh_table): element-to-node table (caller's), the node ->
  // (element, local node) CSR map of its transpose, the element vectors, element groups
  bool table = false;
  const int32_t* conn = nullptr;
  int64_t n_elem = 0;
  int n_groups = 0;
  int32_t* d_csr_off = nullptr;
  int32_t* d_csr_ent = nullptr;
  double* d_evec = nullptr;
  int* d_flag = nullptr;      // [0] non-physical point, [1] phase id outside the table
  double* scratch = nullptr;  // device address of this device's static scratch (pf_apply_adjoint_noalloc)
  bool colours_only = false;  // set while an allocation-free call runs: no brick buffer
  hipStream_t last_stream = nullptr;
  // pf_set_params: pinned staging slots, each reused once its last copy has run
  static constexpr int PARAM_RING = 4;
  struct ParamSlot {
    MatParams<double>* h64 = nullptr;
    MatParams<float>* h32 = nullptr;
    hipEvent_t ev = nullptr;
    bool used = false;
  } pslot[PARAM_RING];
  int pnext = 0;
  MGState mg;
  // multigrid level orders (fine first); n_orders = 0 means p, p-1, ..., 1
  int orders[pfmf::MG_MAX_LEVELS] = {};
  int n_orders = 0;
  // Dirichlet faces (multigrid and Newton step)
  DirMask dir{{0, 0, 0, 0, 0, 0}};
  bool has_dir = false;
  // Newton step workspace: Krylov basis V[m+1], preconditioned vectors Z[m], residual,
  // update; reduction partials; coefficients; FP32 right-hand side and correction
  double* kry = nullptr;
  int kry_m = 0;
  double* kpart = nullptr;
  double* kcoef = nullptr;
  float* k32 = nullptr;
};

// PF_OPT_SCATTER: brick buffer (order 4: element vectors) unless colours were asked for,
// or the automatic choice meets a buffer above PF_SCATTER_AUTO_BYTES; never inside an
// allocation-free call
inline bool use_brick_buffer(const pf_ctx* c) {
  if (c->colours_only) return false;
  if (c->scatter_mode != 0) return c->scatter_mode == 2;
  const int64_t bytes = c->mesh.p == 4 ? (int64_t)c->mesh.nx * c->mesh.ny * c->mesh.nz * 4 * 125 * 8
                                       : (int64_t)c->n_bricks * 4 * 343 * 8;
  return bytes <= PF_SCATTER_AUTO_BYTES;
}

// FP64 residual (MODE 0), Jacobian (1) or adjoint (2) over the context's mesh: every
// launch of one apply on stream s (defined in pf_dispatch.hpp, instantiated once per mode).
template <int MODE>
pf_status dispatch_op64(pf_ctx* c, pfmf::OpArgs a, hipStream_t s);
extern template pf_status dispatch_op64<pfmf::M_RES>(pf_ctx*, pfmf::OpArgs, hipStream_t);
extern template pf_status dispatch_op64<pfmf::M_JAC>(pf_ctx*, pfmf::OpArgs, hipStream_t);
extern template pf_status dispatch_op64<pfmf::M_ADJ>(pf_ctx*, pfmf::OpArgs, hipStream_t);
