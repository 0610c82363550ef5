// libpfmf: host side of the C ABI declared in include/pfmf.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pf_host.hpp"
#include "pf_mfma.hpp"
#include "pf_q4.hpp"
#include "pf_ebe.hpp"
#include "pf_tables.hpp"

using namespace pfmf;

// Scratch of pf_apply_adjoint_noalloc: the per-brick (order 4: per-element) parameter
// partials, PF_NOALLOC_PARTIALS doubles. Every GPU the library runs on holds its own copy
// for the life of the process. In host code `scratch` is only a symbol: its device address
// is taken with hipGetSymbolAddress once per device (noalloc_scratch below) and used
// wherever host code hands the array to a kernel.
static __device__ __align__(256) double scratch[PF_NOALLOC_PARTIALS];

namespace {

thread_local std::string g_err;

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};

}  // namespace

pf_status fail(pf_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

namespace {

MeshDev mesh_dev(const pf_ctx* c) {
  MeshDev m;
  m.nx = c->mesh.nx;
  m.ny = c->mesh.ny;
  m.nz = c->mesh.nz;
  m.nbx = c->nbx;
  m.nby = c->nby;
  m.nbz = c->nbz;
  m.hx = c->mesh.lx / c->mesh.nx;
  m.hy = c->mesh.ly / c->mesh.ny;
  m.hz = c->mesh.lz / c->mesh.nz;
  m.ih[0] = 2.0 / m.hx;
  m.ih[1] = 2.0 / m.hy;
  m.ih[2] = 2.0 / m.hz;
  m.jdet = m.hx * m.hy * m.hz * 0.125;
  return m;
}

template <typename T>
FracParams<T> frac_params(const pf_fracture& f) {
  FracParams<T> r;
  const double c0 = (f.at == 2) ? 2.0 : 8.0 / 3.0;
  r.l0 = (T)f.l0;
  r.eta = (T)f.eta;
  r.zeta = (T)f.zeta;
  r.inv_dt = (T)(1.0 / f.dt);
  r.s_phi = (T)f.s_phi;
  r.c0 = (T)c0;
  r.inv_c0l0 = (T)(1.0 / (c0 * f.l0));
  r.kf = (T)(f.s_phi * 2.0 * f.l0 / c0);
  r.at = f.at;
  return r;
}

template <typename T>
MatParams<T> mat_params(const pf_phase& p, const pf_fracture& f) {
  MatParams<T> m;
  m.mu = (T)(p.E / (2.0 * (1.0 + p.nu)));
  m.kappa = (T)(p.E / (3.0 * (1.0 - 2.0 * p.nu)));
  m.Gc = (T)p.Gc;
  m.sigma0 = (T)p.sigma0;
  m.H = (T)p.H;
  m.a = (T)(p.visc / f.dt);
  m.plastic = p.plastic ? 1 : 0;
  m.sinf = (T)p.sigma_inf;
  m.bv = (T)p.voce_beta;
  m.am = (T)0;
  return m;
}

// Device material of an extra branch (its own spring; Prandtl and Maxwell parameters).
MatParams<double> branch_params(const pf_branch& b, const pf_fracture& f, double Gc) {
  MatParams<double> m{};
  m.mu = b.E / (2.0 * (1.0 + b.nu));
  m.kappa = b.E / (3.0 * (1.0 - 2.0 * b.nu));
  m.Gc = Gc;
  if (b.kind == PF_BRANCH_PRANDTL) {
    m.plastic = 1;
    m.sigma0 = b.sigma0;
    m.H = b.H;
    m.a = b.visc / f.dt;
    m.sinf = b.sigma_inf;
    m.bv = b.voce_beta;
  } else if (b.kind == PF_BRANCH_MAXWELL) {
    m.am = m.mu * f.dt / b.eta_d;
  }
  return m;
}

pf_status upload_mats(pf_ctx* c) {
  std::vector<MatParams<double>> md;
  std::vector<MatParams<float>> mf;
  for (auto& p : c->phases) {
    md.push_back(mat_params<double>(p, c->fr));
    mf.push_back(mat_params<float>(p, c->fr));
  }
  HIPCHK(hipMemcpy(c->d_mats, md.data(), md.size() * sizeof(md[0]), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(c->d_matsf, mf.data(), mf.size() * sizeof(mf[0]), hipMemcpyHostToDevice));
  return PF_OK;
}

// Stream-ordered upload of the material tables: the tables are written into a pinned
// staging slot and copied on stream s, so applies enqueued before the call on s read the
// old values and later ones the new. A slot is rewritten only after its previous copy
// ran (an event per slot; the host waits only when PARAM_RING uploads are still queued).
pf_status upload_mats_async(pf_ctx* c, hipStream_t s) {
  const size_t nph = c->phases.size();
  pf_ctx::ParamSlot& ps = c->pslot[c->pnext];
  if (!ps.h64) {
    if (hipHostMalloc((void**)&ps.h64, nph * sizeof(MatParams<double>), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&ps.h32, nph * sizeof(MatParams<float>), hipHostMallocDefault) != hipSuccess)
      return fail(PF_ENOMEM, "pinned parameter staging: allocation failed");
    HIPCHK(hipEventCreateWithFlags(&ps.ev, hipEventDisableTiming));
  } else if (ps.used) {
    HIPCHK(hipEventSynchronize(ps.ev));
  }
  for (size_t i = 0; i < nph; ++i) {
    ps.h64[i] = mat_params<double>(c->phases[i], c->fr);
    ps.h32[i] = mat_params<float>(c->phases[i], c->fr);
  }
  HIPCHK(hipMemcpyAsync(c->d_mats, ps.h64, nph * sizeof(MatParams<double>), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(c->d_matsf, ps.h32, nph * sizeof(MatParams<float>), hipMemcpyHostToDevice, s));
  HIPCHK(hipEventRecord(ps.ev, s));
  ps.used = true;
  c->pnext = (c->pnext + 1) % pf_ctx::PARAM_RING;
  return PF_OK;
}

pf_status build_tables(pf_ctx* c) {
  auto* t = new DevTables;
  auto* tf = new DevTablesF;
  std::memset(t, 0, sizeof *t);
  std::memset(tf, 0, sizeof *tf);
  for (int P = 2; P <= 5; ++P) {
    std::vector<double> xn;
    gauss_lobatto(P, xn);
    for (int Q = 2; Q <= 5; ++Q) {
      std::vector<double> xq, wq, B, D;
      gauss_legendre(Q, xq, wq);
      lagrange_tables(xn, xq, B, D);
      std::vector<double> Bg, Gg;
      lagrange_tables(xq, xq, Bg, Gg);
      for (int q = 0; q < Q; ++q) {
        t->w[Q][q] = wq[q];
        tf->w[Q][q] = (float)wq[q];
        for (int m = 0; m < Q; ++m) {
          t->G[Q][q][m] = Gg[q * Q + m];
          tf->G[Q][q][m] = (float)Gg[q * Q + m];
        }
        for (int i = 0; i < P; ++i) {
          t->B[P][Q][q][i] = B[q * P + i];
          t->D[P][Q][q][i] = D[q * P + i];
          tf->B[P][Q][q][i] = (float)B[q * P + i];
          tf->D[P][Q][q][i] = (float)D[q * P + i];
        }
      }
    }
  }
  hipError_t e1 = hipMalloc(&c->d_tab, sizeof(DevTables));
  hipError_t e2 = hipMalloc(&c->d_tabf, sizeof(DevTablesF));
  if (e1 != hipSuccess || e2 != hipSuccess) {
    delete t;
    delete tf;
    return fail(PF_ENOMEM, "table allocation failed");
  }
  hipError_t e3 = hipMemcpy(c->d_tab, t, sizeof(DevTables), hipMemcpyHostToDevice);
  hipError_t e4 = hipMemcpy(c->d_tabf, tf, sizeof(DevTablesF), hipMemcpyHostToDevice);
  delete t;
  delete tf;
  if (e3 != hipSuccess || e4 != hipSuccess) return fail(PF_EHIP, "table upload failed");
  return PF_OK;
}

pf_status check_ctx(pf_ctx* c) {
  if (!c) return fail(PF_EINVAL, "null context");
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev != c->device) return fail(PF_EINVAL, "context belongs to device %d, current device is %d", c->device, dev);
  return PF_OK;
}

OpArgs op_args(pf_ctx* c) {
  OpArgs a;
  a.m = mesh_dev(c);
  a.nx1 = c->nx1;
  a.ny1 = c->ny1;
  a.n_nodes = c->n_nodes;
  a.n_q = c->n_q;
  a.z = nullptr;
  a.w = nullptr;
  a.phin = c->phi_n;
  a.state = c->qp_state;
  a.phase = c->qp_phase;
  a.mats = c->d_mats;
  a.nph = (int)c->phases.size();
  a.fr = frac_params<double>(c->fr);
  a.out = nullptr;
  a.gpart = c->d_gpart;
  a.ebuf = nullptr;
  a.brick_base = 0;
  a.flag = c->d_flag;
  a.xb = c->d_xb;
  a.xstate = c->xstate;
  a.n_extra = c->n_extra;
  a.qd = c->d_qd;
  a.conn = c->conn;
  a.n_elem = c->n_elem;
  a.evec = c->d_evec;
  a.n_groups = c->n_groups;
  return a;
}

// Calls that need the box lattice refuse a table-restriction context.
pf_status box_only(const pf_ctx* c, const char* what) {
  if (c->table) return fail(PF_EUNSUPPORTED, "%s needs the box lattice (the context has a table restriction)", what);
  return PF_OK;
}

// Device address of the static scratch on device dev (current), taken once per device.
pf_status noalloc_scratch(int dev, double** out) {
  if (dev < 0 || dev >= MAX_DEVICES) return fail(PF_EUNSUPPORTED, "device %d outside 0..%d", dev, MAX_DEVICES - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail(PF_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return PF_OK;
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + nb && pb < pa + na;
}

}  // namespace

extern "C" {

const char* pf_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace {

// Checks shared by both setup calls: phases, fracture parameters.
pf_status check_materials(const pf_phase* phases, int n_phases, const pf_fracture* fr) {
  if (n_phases < 1 || n_phases > 255) return fail(PF_EINVAL, "n_phases=%d outside 1..255", n_phases);
  if (!(fr->l0 > 0 && fr->dt > 0 && fr->eta >= 0 && fr->s_phi > 0) || (fr->at != 1 && fr->at != 2))
    return fail(PF_EINVAL, "bad fracture parameters");
  for (int i = 0; i < n_phases; ++i) {
    const pf_phase& p = phases[i];
    if (!(p.E > 0 && p.nu > -1 && p.nu < 0.5 && p.Gc >= 0 && p.sigma0 >= 0 && p.H >= 0 && p.visc >= 0))
      return fail(PF_EINVAL, "bad parameters for phase %d", i);
    if (p.plastic && !(p.sigma0 > 0)) return fail(PF_EINVAL, "plastic phase %d needs sigma0 > 0", i);
    if (!(p.voce_beta >= 0) || (p.voce_beta > 0 && !(p.sigma_inf >= p.sigma0)))
      return fail(PF_EINVAL, "phase %d: Voce needs voce_beta >= 0 and sigma_inf >= sigma0", i);
  }
  return PF_OK;
}

// The rest of a context once its sizes are set: tables, materials, partials, flags and
// the check of the phase ids (stream-ordered after the caller's writes; synchronises).
pf_status setup_common(pf_ctx* c, const pf_phase* phases, int n_phases, const pf_fracture* fr,
                       const uint8_t* qp_phase, const double* qp_state, const double* phi_n, void* stream) {
  c->phases.assign(phases, phases + n_phases);
  for (int i = 0; i < n_phases; ++i) c->has_voce |= phases[i].plastic && phases[i].voce_beta > 0;
  c->fr = *fr;
  c->qp_phase = qp_phase;
  c->qp_state = qp_state;
  c->phi_n = phi_n;
  c->last_stream = (hipStream_t)stream;
  pf_status st = build_tables(c);
  if (st != PF_OK) return st;
  if (hipMalloc(&c->d_mats, n_phases * sizeof(MatParams<double>)) != hipSuccess ||
      hipMalloc(&c->d_matsf, n_phases * sizeof(MatParams<float>)) != hipSuccess ||
      hipMalloc(&c->d_gpart, (size_t)c->n_parts * n_phases * 3 * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->d_flag, 2 * sizeof(int)) != hipSuccess)
    return fail(PF_ENOMEM, "context allocation failed");
  if (hipMemset(c->d_flag, 0, 2 * sizeof(int)) != hipSuccess) return fail(PF_EHIP, "memset failed");
  st = upload_mats(c);
  if (st != PF_OK) return st;
  st = noalloc_scratch(c->device, &c->scratch);
  if (st != PF_OK) return st;
  const hipStream_t s = (hipStream_t)stream;
  int bad = 0;
  hipLaunchKernelGGL(k_check_phase, dim3((unsigned)std::min<int64_t>((c->n_q + NT - 1) / NT, 4096)), dim3(NT), 0, s,
                     qp_phase, c->n_q, n_phases, c->d_flag);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(&bad, c->d_flag + 1, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(PF_EHIP, "phase check: %s", hipGetErrorString(e));
  if (bad) return fail(PF_EINVAL, "qp_phase holds an id >= n_phases (%d)", n_phases);
  return PF_OK;
}

}  // namespace

extern "C" {

pf_status pf_setup_mesh(const pf_mesh_desc* mesh, const pf_phase* phases, int n_phases, const pf_fracture* fr,
                        const uint8_t* qp_phase, const double* qp_state, const double* phi_n, void* stream,
                        pf_ctx** out) {
  g_err.clear();
  if (!out) return fail(PF_EINVAL, "out is null");
  *out = nullptr;
  if (!mesh || !phases || !fr || !qp_phase || !qp_state || !phi_n) return fail(PF_EINVAL, "null argument");
  if (mesh->p < 1 || mesh->p > 4) return fail(PF_EUNSUPPORTED, "order p=%d outside 1..4", mesh->p);
  if (mesh->nx < 1 || mesh->ny < 1 || mesh->nz < 1) return fail(PF_EINVAL, "empty mesh");
  if (!(mesh->lx > 0 && mesh->ly > 0 && mesh->lz > 0)) return fail(PF_EINVAL, "box lengths must be positive");
  pf_status st0 = check_materials(phases, n_phases, fr);
  if (st0) return st0;
  const int64_t nx1 = (int64_t)mesh->p * mesh->nx + 1, ny1 = (int64_t)mesh->p * mesh->ny + 1,
                nz1 = (int64_t)mesh->p * mesh->nz + 1;
  if (nx1 * ny1 * nz1 >= (int64_t)1 << 31) return fail(PF_EINVAL, "mesh too large for 32-bit node ids");
  auto* c = new pf_ctx;
  (void)hipGetDevice(&c->device);
  c->mesh = *mesh;
  c->P = mesh->p + 1;
  c->Q = mesh->p + 1;
  c->nx1 = (int)nx1;
  c->ny1 = (int)ny1;
  c->nz1 = (int)nz1;
  c->n_nodes = nx1 * ny1 * nz1;
  c->n_q = (int64_t)mesh->nx * mesh->ny * mesh->nz * c->Q * c->Q * c->Q;
  c->nbx = (mesh->nx + 1) / 2;
  c->nby = (mesh->ny + 1) / 2;
  c->nbz = (mesh->nz + 1) / 2;
  c->n_bricks = c->nbx * c->nby * c->nbz;
  // adjoint parameter partials: one slot per brick, or per element for order 4
  c->n_parts = mesh->p == 4 ? mesh->nx * mesh->ny * mesh->nz : c->n_bricks;
  c->colour_base[0] = 0;
  for (int col = 0; col < 8; ++col)
    c->colour_base[col + 1] = c->colour_base[col] + bricks_in_colour(c->nbx, c->nby, c->nbz, col);
  pf_status st = setup_common(c, phases, n_phases, fr, qp_phase, qp_state, phi_n, stream);
  if (st != PF_OK) { pf_destroy(c); return st; }
  *out = c;
  return PF_OK;
}

pf_status pf_setup_mesh_table(const pf_table_mesh_desc* mesh, const int32_t* conn, const double* X,
                              const pf_phase* phases, int n_phases, const pf_fracture* fr, const uint8_t* qp_phase,
                              const double* qp_state, const double* phi_n, void* stream, pf_ctx** out) {
  g_err.clear();
  if (!out) return fail(PF_EINVAL, "out is null");
  *out = nullptr;
  if (!mesh || !conn || !X || !phases || !fr || !qp_phase || !qp_state || !phi_n) return fail(PF_EINVAL, "null argument");
  if (mesh->p < 2 || mesh->p > 4) return fail(PF_EUNSUPPORTED, "table restriction built for p = 2..4 (p=%d)", mesh->p);
  const int P = mesh->p + 1, P3 = P * P * P;
  if (mesh->n_elem < 1 || mesh->n_nodes < 1) return fail(PF_EINVAL, "empty mesh");
  if (mesh->n_nodes >= ((int64_t)1 << 31) - 1 || mesh->n_elem * 4 * P3 >= ((int64_t)1 << 31))
    return fail(PF_EINVAL, "mesh too large for 32-bit node and element-vector indices");
  pf_status st0 = check_materials(phases, n_phases, fr);
  if (st0) return st0;
  const hipStream_t s = (hipStream_t)stream;
  // the table on the host: range check and the CSR map of its transpose (node -> entries
  // (e P^3 + a) 4 in element order), built once here
  std::vector<int32_t> h((size_t)mesh->n_elem * P3);
  {
    hipError_t e = hipMemcpyAsync(h.data(), conn, h.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(PF_EHIP, "reading the element table: %s", hipGetErrorString(e));
  }
  std::vector<int32_t> off((size_t)mesh->n_nodes + 1, 0), ent(h.size());
  for (size_t k = 0; k < h.size(); ++k) {
    if (h[k] < 0 || h[k] >= mesh->n_nodes)
      return fail(PF_EINVAL, "element %lld, local node %d: node %d outside 0..%lld", (long long)(k / P3), (int)(k % P3),
                  h[k], (long long)mesh->n_nodes - 1);
    ++off[(size_t)h[k] + 1];
  }
  for (int64_t i = 0; i < mesh->n_nodes; ++i) off[i + 1] += off[i];
  {
    std::vector<int32_t> fill(off.begin(), off.end() - 1);
    for (size_t k = 0; k < h.size(); ++k) {
      const int64_t e = (int64_t)(k / P3), a = (int64_t)(k % P3);
      ent[fill[h[k]]++] = (int32_t)((e * P3 + a) * 4);
    }
  }
  auto* c = new pf_ctx;
  (void)hipGetDevice(&c->device);
  c->table = true;
  c->mesh = pf_mesh_desc{mesh->p, 0, 0, 0, 1.0, 1.0, 1.0};
  c->P = P;
  c->Q = P;
  c->n_nodes = mesh->n_nodes;
  c->n_elem = mesh->n_elem;
  c->n_q = mesh->n_elem * P3;
  // workgroups: 8 elements each on orders 2 and 3 (two per wave), one element on order 4
  c->n_groups = mesh->p == 4 ? (int)mesh->n_elem : (int)((mesh->n_elem + 7) / 8);
  c->n_parts = c->n_groups;
  c->conn = conn;
  pf_status st = setup_common(c, phases, n_phases, fr, qp_phase, qp_state, phi_n, stream);
  if (st != PF_OK) { pf_destroy(c); return st; }
  if (hipMalloc(&c->d_csr_off, off.size() * sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&c->d_csr_ent, ent.size() * sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&c->d_evec, (size_t)c->n_elem * 4 * P3 * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->d_qd, (size_t)GEO_N * c->n_q * sizeof(double)) != hipSuccess) {
    pf_destroy(c);
    return fail(PF_ENOMEM, "table restriction: allocation failed");
  }
  hipError_t e = hipMemcpyAsync(c->d_csr_off, off.data(), off.size() * sizeof(int32_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(c->d_csr_ent, ent.data(), ent.size() * sizeof(int32_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(c->d_flag, 0, 2 * sizeof(int), s);
  if (e == hipSuccess) {
    const dim3 grid((unsigned)((c->n_q + NT - 1) / NT));
    if (mesh->p == 2)
      hipLaunchKernelGGL((k_geometry_tab<3, 3>), grid, dim3(NT), 0, s, X, c->n_nodes, conn, c->n_q, c->d_tab, c->d_qd,
                         c->d_flag);
    else if (mesh->p == 3)
      hipLaunchKernelGGL((k_geometry_tab<4, 4>), grid, dim3(NT), 0, s, X, c->n_nodes, conn, c->n_q, c->d_tab, c->d_qd,
                         c->d_flag);
    else
      hipLaunchKernelGGL((k_geometry_tab<5, 5>), grid, dim3(NT), 0, s, X, c->n_nodes, conn, c->n_q, c->d_tab, c->d_qd,
                         c->d_flag);
    e = hipGetLastError();
  }
  int bad = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&bad, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // also keeps off / ent alive until copied
  if (e != hipSuccess) { pf_destroy(c); return fail(PF_EHIP, "table setup: %s", hipGetErrorString(e)); }
  if (bad) {
    (void)hipMemset(c->d_flag, 0, 2 * sizeof(int));
    pf_destroy(c);
    return fail(PF_EINVAL, "node positions give an element with det J <= 0 at some quadrature point");
  }
  *out = c;
  return PF_OK;
}

pf_status pf_sizes(const pf_ctx* c, int64_t* n_nodes, int64_t* n_q, int64_t* n_dof) {
  if (!c) return fail(PF_EINVAL, "null context");
  if (n_nodes) *n_nodes = c->n_nodes;
  if (n_q) *n_q = c->n_q;
  if (n_dof) *n_dof = 4 * c->n_nodes;
  return PF_OK;
}

pf_status pf_set_branches(pf_ctx* c, const pf_branch* branches, int n_extra, const double* xstate) {
  pf_status st = check_ctx(c);
  if (st) return st;
  if ((st = box_only(c, "pf_set_branches"))) return st;
  if (n_extra < 0 || n_extra > PF_MAX_EXTRA_BRANCHES)
    return fail(PF_EINVAL, "n_extra=%d outside 0..%d", n_extra, PF_MAX_EXTRA_BRANCHES);
  if (n_extra > 0 && (!branches || !xstate)) return fail(PF_EINVAL, "null branches or xstate");
  if (n_extra > 0 && c->mesh.p < 2) return fail(PF_EUNSUPPORTED, "extra branches need p >= 2");
  const int nph = (int)c->phases.size();
  std::vector<XBranch> xb((size_t)nph * (n_extra > 0 ? n_extra : 1));
  for (int i = 0; i < nph * n_extra; ++i) {
    const pf_branch& b = branches[i];
    if (b.kind < PF_BRANCH_NONE || b.kind > PF_BRANCH_PRANDTL) return fail(PF_EINVAL, "branch %d: bad kind %d", i, b.kind);
    xb[i].kind = b.kind;
    xb[i].m = MatParams<double>{};
    if (b.kind == PF_BRANCH_NONE) continue;
    if (!(b.E > 0) || !(b.nu > -1.0 && b.nu < 0.5)) return fail(PF_EINVAL, "branch %d: bad E or nu", i);
    if (b.kind == PF_BRANCH_MAXWELL && !(b.eta_d > 0)) return fail(PF_EINVAL, "branch %d: Maxwell needs eta_d > 0", i);
    if (b.kind == PF_BRANCH_PRANDTL) {
      if (!(b.sigma0 > 0 && b.H >= 0 && b.visc >= 0 && b.voce_beta >= 0))
        return fail(PF_EINVAL, "branch %d: bad Prandtl parameters", i);
      if (b.voce_beta > 0 && !(b.sigma_inf >= b.sigma0))
        return fail(PF_EINVAL, "branch %d: Voce needs sigma_inf >= sigma0", i);
    }
    xb[i].m = branch_params(b, c->fr, c->phases[i / n_extra].Gc);
  }
  std::vector<MatParams<double>> x64(xb.size());
  std::vector<MatParams<float>> x32(xb.size());
  for (size_t i = 0; i < xb.size(); ++i) {
    const MatParams<double>& m = xb[i].m;
    x64[i] = m;
    x32[i] = MatParams<float>{(float)m.mu, (float)m.kappa, (float)m.Gc, (float)m.sigma0, (float)m.H, (float)m.a,
                              m.plastic, (float)m.sinf, (float)m.bv, (float)m.am};
  }
  HIPCHK(hipDeviceSynchronize());  // applies in flight may still read the old tables
  (void)hipFree(c->d_xb);
  (void)hipFree(c->d_xmats64);
  (void)hipFree(c->d_xmatsf);
  c->d_xb = nullptr;
  c->d_xmats64 = nullptr;
  c->d_xmatsf = nullptr;
  c->n_extra = 0;
  c->xvoce = false;
  c->xstate = nullptr;
  if (n_extra > 0) {
    if (hipMalloc(&c->d_xb, xb.size() * sizeof(XBranch)) != hipSuccess ||
        hipMalloc(&c->d_xmats64, x64.size() * sizeof(x64[0])) != hipSuccess ||
        hipMalloc(&c->d_xmatsf, x32.size() * sizeof(x32[0])) != hipSuccess)
      return fail(PF_ENOMEM, "branch table allocation failed");
    HIPCHK(hipMemcpy(c->d_xb, xb.data(), xb.size() * sizeof(XBranch), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->d_xmats64, x64.data(), x64.size() * sizeof(x64[0]), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->d_xmatsf, x32.data(), x32.size() * sizeof(x32[0]), hipMemcpyHostToDevice));
    c->n_extra = n_extra;
    c->xstate = xstate;
    for (int i = 0; i < nph * n_extra; ++i)
      c->xvoce |= branches[i].kind == PF_BRANCH_PRANDTL && branches[i].voce_beta > 0;
  }
  c->mg.linearized = false;  // the linearisation covers the single block
  c->mg.lin64_valid = false;
  return PF_OK;
}

pf_status pf_set_params(pf_ctx* c, const double* params, void* stream) {
  pf_status st = check_ctx(c);
  if (st) return st;
  if (!params) return fail(PF_EINVAL, "null params");
  for (size_t i = 0; i < c->phases.size(); ++i) {
    const double gc = params[3 * i], s0 = params[3 * i + 1], vi = params[3 * i + 2];
    if (!(gc >= 0 && s0 >= 0 && vi >= 0)) return fail(PF_EINVAL, "bad parameters for phase %zu", i);
    if (c->phases[i].plastic && !(s0 > 0)) return fail(PF_EINVAL, "plastic phase %zu needs sigma0 > 0", i);
    if (c->phases[i].voce_beta > 0 && !(c->phases[i].sigma_inf >= s0))
      return fail(PF_EINVAL, "phase %zu: Voce needs sigma_inf >= sigma0", i);
  }
  bool same = true;
  for (size_t i = 0; i < c->phases.size(); ++i)
    same = same && c->phases[i].Gc == params[3 * i] && c->phases[i].sigma0 == params[3 * i + 1] &&
           c->phases[i].visc == params[3 * i + 2];
  if (same) return PF_OK;  // nothing to upload; the linearisation stays valid
  c->mg.linearized = false;  // the records hold decisions taken with the old parameters
  c->mg.lin64_valid = false;
  for (size_t i = 0; i < c->phases.size(); ++i) {
    c->phases[i].Gc = params[3 * i];
    c->phases[i].sigma0 = params[3 * i + 1];
    c->phases[i].visc = params[3 * i + 2];
  }
  c->last_stream = (hipStream_t)stream;
  return upload_mats_async(c, (hipStream_t)stream);
}

pf_status pf_apply_residual(pf_ctx* c, const double* z, double* r, void* stream) {
  pf_status st = check_ctx(c);
  if (st) return st;
  if (!z || !r) return fail(PF_EINVAL, "null vector");
  const size_t nb = 4 * c->n_nodes * sizeof(double);
  if (overlaps(z, nb, r, nb)) return fail(PF_EINVAL, "r aliases z");
  OpArgs a = op_args(c);
  a.z = z;
  a.out = r;
  c->last_stream = (hipStream_t)stream;
  return dispatch_op64<M_RES>(c, a, (hipStream_t)stream);
}

pf_status pf_apply_jacobian(pf_ctx* c, const double* z, const double* dz, double* y, void* stream) {
  pf_status st = check_ctx(c);
  if (st) return st;
  if (!z || !dz || !y) return fail(PF_EINVAL, "null vector");
  const size_t nb = 4 * c->n_nodes * sizeof(double);
  if (overlaps(z, nb, y, nb) || overlaps(dz, nb, y, nb)) return fail(PF_EINVAL, "y aliases an input");
  OpArgs a = op_args(c);
  a.z = z;
  a.w = dz;
  a.out = y;
  c->last_stream = (hipStream_t)stream;
  return dispatch_op64<M_JAC>(c, a, (hipStream_t)stream);
}

pf_status pf_apply_adjoint(pf_ctx* c, const double* z, const double* v, double* gz, double* gparams, void* stream) {
  pf_status st = check_ctx(c);
  if (st) return st;
  if (!z || !v || !gz || !gparams) return fail(PF_EINVAL, "null vector");
  const size_t nb = 4 * c->n_nodes * sizeof(double);
  const size_t np = c->phases.size() * 3 * sizeof(double);
  if (overlaps(z, nb, gz, nb) || overlaps(v, nb, gz, nb) || overlaps(gparams, np, gz, nb) ||
      overlaps(gparams, np, z, nb) || overlaps(gparams, np, v, nb))
    return fail(PF_EINVAL, "an output aliases an input");
  OpArgs a = op_args(c);
  a.z = z;
  a.w = v;
  a.out = gz;
  c->last_stream = (hipStream_t)stream;
  st = dispatch_op64<M_ADJ>(c, a, (hipStream_t)stream);
  if (st) return st;
  hipLaunchKernelGGL(k_sum_params, dim3((int)c->phases.size() * 3), dim3(NT), 0, (hipStream_t)stream, c->d_gpart,
                     c->n_parts, (int)c->phases.size(), gparams);
  HIPCHK(hipGetLastError());
  return PF_OK;
}

pf_status pf_apply_adjoint_noalloc(pf_ctx* c, const double* z, const double* v, double* gz, double* gparams,
                                   void* stream) {
  pf_status st = check_ctx(c);
  if (st) return st;
  if ((st = box_only(c, "pf_apply_adjoint_noalloc"))) return st;
  if (!z || !v || !gz || !gparams) return fail(PF_EINVAL, "null vector");
  const int64_t nparts = (int64_t)c->n_parts * (int64_t)c->phases.size() * 3;
  if (nparts > PF_NOALLOC_PARTIALS)
    return fail(PF_EINVAL, "%lld parameter partials exceed the allocation-free scratch (%d doubles)",
                (long long)nparts, PF_NOALLOC_PARTIALS);
  if (!c->scratch) return fail(PF_EHIP, "no scratch address for device %d", c->device);
  const size_t nb = 4 * c->n_nodes * sizeof(double);
  const size_t np = c->phases.size() * 3 * sizeof(double);
  if (overlaps(z, nb, gz, nb) || overlaps(v, nb, gz, nb) || overlaps(gparams, np, gz, nb) ||
      overlaps(gparams, np, z, nb) || overlaps(gparams, np, v, nb))
    return fail(PF_EINVAL, "an output aliases an input");
  OpArgs a = op_args(c);
  a.z = z;
  a.w = v;
  a.out = gz;
  a.gpart = c->scratch;  // every brick (element) slot is written by the apply: nothing to clear
  c->last_stream = (hipStream_t)stream;
  c->colours_only = true;
  st = dispatch_op64<M_ADJ>(c, a, (hipStream_t)stream);
  c->colours_only = false;
  if (st) return st;
  hipLaunchKernelGGL(k_sum_params, dim3((int)c->phases.size() * 3), dim3(NT), 0, (hipStream_t)stream, c->scratch,
                     c->n_parts, (int)c->phases.size(), gparams);
  HIPCHK(hipGetLastError());
  return PF_OK;
}

pf_status pf_set_option(pf_ctx* c, int option, int value) {
  pf_status st = check_ctx(c);
  if (st) return st;
  switch (option) {
    case PF_OPT_SCATTER:
      if (value < 0 || value > 2) return fail(PF_EINVAL, "PF_OPT_SCATTER takes 0, 1 or 2, not %d", value);
      c->scatter_mode = value;
      return PF_OK;
    case PF_OPT_STORE_LIN64:
      if (value < 0 || value > 1) return fail(PF_EINVAL, "PF_OPT_STORE_LIN64 takes 0 or 1, not %d", value);
      c->store_lin64 = value != 0;
      c->mg.lin64_valid = false;
      return PF_OK;
    default:
      return fail(PF_EINVAL, "unknown option %d", option);
  }
}

pf_status pf_check(pf_ctx* c) {
  pf_status st = check_ctx(c);
  if (st) return st;
  HIPCHK(hipStreamSynchronize(c->last_stream));
  int flag[2] = {0, 0};
  HIPCHK(hipMemcpy(flag, c->d_flag, 2 * sizeof(int), hipMemcpyDeviceToHost));
  if (flag[0] || flag[1]) {
    HIPCHK(hipMemset(c->d_flag, 0, 2 * sizeof(int)));
    if (flag[1]) return fail(PF_EINVAL, "a quadrature point holds a phase id >= n_phases");
    return fail(PF_ENONPHYSICAL, "a quadrature point left the physical domain (det F <= 0 or b_i <= 0)");
  }
  return PF_OK;
}

pf_status pf_set_geometry(pf_ctx* c, const double* X, void* stream) {
  pf_status st = check_ctx(c);
  if (st) return st;
  if ((st = box_only(c, "pf_set_geometry"))) return st;
  hipStream_t s = (hipStream_t)stream;
  if (X && (c->mesh.p < 2 || c->mesh.p > 4))
    return fail(PF_EUNSUPPORTED, "mapped elements are built for p = 2..4 (p=%d)", c->mesh.p);
  HIPCHK(hipDeviceSynchronize());  // applies in flight may still read the old record
  (void)hipFree(c->d_qd);
  (void)hipFree(c->d_qd32);
  c->d_qd = nullptr;
  c->d_qd32 = nullptr;
  c->mg.linearized = false;  // a linearisation belongs to the geometry it was taken on
  c->mg.lin64_valid = false;
  if (!X) return PF_OK;
  double* qd = nullptr;
  int* flag = nullptr;
  if (hipMalloc(&qd, (size_t)GEO_N * c->n_q * sizeof(double)) != hipSuccess) return fail(PF_ENOMEM, "geometry record: allocation failed");
  if (hipMalloc(&flag, sizeof(int)) != hipSuccess) {
    (void)hipFree(qd);
    return fail(PF_ENOMEM, "geometry flag: allocation failed");
  }
  int bad = 0;
  hipError_t e = hipMemsetAsync(flag, 0, sizeof(int), s);
  if (e == hipSuccess) {
    const dim3 grid((unsigned)((c->n_q + NT - 1) / NT));
    const DevTables* tab = c->d_tab;
    if (c->mesh.p == 2)
      hipLaunchKernelGGL((k_geometry<3, 3>), grid, dim3(NT), 0, s, X, c->n_nodes, c->nx1, c->ny1, c->mesh.nx,
                         c->mesh.ny, c->n_q, tab, qd, flag);
    else if (c->mesh.p == 3)
      hipLaunchKernelGGL((k_geometry<4, 4>), grid, dim3(NT), 0, s, X, c->n_nodes, c->nx1, c->ny1, c->mesh.nx,
                         c->mesh.ny, c->n_q, tab, qd, flag);
    else
      hipLaunchKernelGGL((k_geometry<5, 5>), grid, dim3(NT), 0, s, X, c->n_nodes, c->nx1, c->ny1, c->mesh.nx,
                         c->mesh.ny, c->n_q, tab, qd, flag);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(flag);
  if (e != hipSuccess) {
    (void)hipFree(qd);
    return fail(PF_EHIP, "geometry setup: %s", hipGetErrorString(e));
  }
  if (bad) {
    (void)hipFree(qd);
    return fail(PF_EINVAL, "node positions give an element with det J <= 0 at some quadrature point");
  }
  float* qd32 = nullptr;
  if (hipMalloc(&qd32, (size_t)GEO_N * c->n_q * sizeof(float)) != hipSuccess) {
    (void)hipFree(qd);
    return fail(PF_ENOMEM, "geometry record (FP32): allocation failed");
  }
  const int64_t nr = (int64_t)GEO_N * c->n_q;
  hipLaunchKernelGGL(k_to_f32, dim3((unsigned)std::min<int64_t>((nr + NT - 1) / NT, 65536)), dim3(NT), 0, s, qd, qd32, nr);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    (void)hipFree(qd);
    (void)hipFree(qd32);
    return fail(PF_EHIP, "geometry setup: %s", hipGetErrorString(e));
  }
  c->d_qd = qd;
  c->d_qd32 = qd32;
  return PF_OK;
}

void pf_destroy(pf_ctx* c) {
  if (!c) return;
  (void)hipDeviceSynchronize();
  mg_free(c->mg);
  (void)hipFree(c->kry);
  (void)hipFree(c->kpart);
  (void)hipFree(c->kcoef);
  (void)hipFree(c->k32);
  (void)hipFree(c->d_tab);
  (void)hipFree(c->d_tabf);
  (void)hipFree(c->d_mats);
  (void)hipFree(c->d_matsf);
  (void)hipFree(c->d_gpart);
  (void)hipFree(c->d_ebuf);
  (void)hipFree(c->d_flag);
  (void)hipFree(c->d_xb);
  (void)hipFree(c->d_xmats64);
  (void)hipFree(c->d_xmatsf);
  (void)hipFree(c->d_qd);
  (void)hipFree(c->d_qd32);
  (void)hipFree(c->d_csr_off);
  (void)hipFree(c->d_csr_ent);
  (void)hipFree(c->d_evec);
  for (auto& ps : c->pslot) {
    (void)hipHostFree(ps.h64);
    (void)hipHostFree(ps.h32);
    if (ps.ev) (void)hipEventDestroy(ps.ev);
  }
  delete c;
}

}  // extern "C"

#include "pf_mg_host.hpp"
#include "pf_newton_host.hpp"
