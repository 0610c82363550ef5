// FP32 p-multigrid: linearisation record, level operators at the fine
// quadrature, point-Jacobi diagonals, level transfers and Chebyshev vector ops.
//
// Levels are orders p, p-1, ..., coarse_p on the same mesh. Every level is
// evaluated at the fine Gauss points with the fine linearisation record, so a
// coarse operator is the Galerkin product P^T A P of the fine one (the coarse
// space is a subspace of the fine space). Below an order-1 level the hierarchy may
// continue on coarser order-1 lattices (every second node per direction, trilinear
// interpolation), each operator the Galerkin product of the one above, formed once
// per linearisation as a block stencil. Kinematics (F, eigenframe, log strains)
// are recomputed in FP32 from FP32 mirrors of u and D at every apply; the yield,
// split and history decisions and the return-mapping scalars come from the
// record taken in FP64 by the linearisation.
#pragma once
#include <hip/hip_runtime.h>

#include "pf_brick.hpp"
#include "pf_ops.hpp"
#include "pf_qf.hpp"
#include "pf_geom.hpp"

namespace pfmf {

template <typename V> struct RecordSoAT {
  V* rec;          // [REC_N][n_q], slots as in LinRecordT
  uint8_t* flags;  // [n_q]
};
using RecordSoA = RecordSoAT<float>;

struct LevelDev {
  int P;           // nodes per direction of this level's elements
  int nx1, ny1;
  int64_t n_nodes;
};

constexpr int MG_MAX_LEVELS = 8;

struct MGLevel {
  int p = 0, P = 0;
  // h: coarsening depth of an order-1 level (0: the mesh itself; h > 0: the order-1
  // lattice with 2^h times fewer elements per direction, its operator the Galerkin
  // product of the finer order-1 level's, stored as a block stencil S)
  int h = 0;
  int ne[3] = {0, 0, 0};  // elements per direction of this level's lattice
  int nx1 = 0, ny1 = 0, nz1 = 0;
  int64_t n_nodes = 0;
  float* S = nullptr;  // h > 0: block stencil [27][4][4][n_nodes]
  float *x = nullptr, *r = nullptr, *d = nullptr, *t = nullptr, *b = nullptr;
  float *diag = nullptr, *dinv = nullptr;
  double lmax = 0.0;
  // transfer to the next coarser level: per direction, prolongation rows
  // (fine index -> coarse base + Pc weights) and restriction rows
  // (coarse index -> fine base + (2 pf + 1) weights)
  int* pbase[3] = {nullptr, nullptr, nullptr};
  float* pw[3] = {nullptr, nullptr, nullptr};
  int* rbase[3] = {nullptr, nullptr, nullptr};
  float* rw[3] = {nullptr, nullptr, nullptr};
};

struct MGState {
  int n_levels = 0;
  MGLevel lv[MG_MAX_LEVELS];
  float* z32 = nullptr;  // FP32 mirror of u on the fine level [3][n_nodes]
  RecordSoA rec{nullptr, nullptr};  // [rec_layers][REC_N][n_q] and flags [rec_layers][n_q]
  float* tmpA = nullptr;
  float* tmpB = nullptr;
  double* red = nullptr;  // reduction scratch
  float* ebe = nullptr;    // element matrices of the order-1 level on the mesh [n_elem][32][32]
  float* stencil = nullptr;  // the same level as a block stencil [27][4][4][n_nodes]
  float* ebuf32 = nullptr;   // brick-buffer scatter of the FP32 level applies
  double* rec64 = nullptr;   // stored FP64 linearisation [rec_layers][REC_N][n_q] (flags in rec.flags)
  double* u64 = nullptr;     // u at the linearisation point [3][n_nodes]
  int rec_layers = 0;        // record layers allocated (1 + extra branches)
  int ebe_level = -1;
  bool linearized = false;
  bool lin64_valid = false;  // rec64 / u64 hold the current linearisation
};

inline void mg_free_level(MGLevel& L) {
  float* fs[] = {L.x, L.r, L.d, L.t, L.b, L.diag, L.dinv, L.S};
  for (float* f : fs) (void)hipFree(f);
  for (int k = 0; k < 3; ++k) {
    (void)hipFree(L.pbase[k]);
    (void)hipFree(L.pw[k]);
    (void)hipFree(L.rbase[k]);
    (void)hipFree(L.rw[k]);
  }
  L = MGLevel();
}

inline void mg_free(MGState& mg) {
  for (int l = 0; l < MG_MAX_LEVELS; ++l) mg_free_level(mg.lv[l]);
  (void)hipFree(mg.z32);
  (void)hipFree(mg.rec.rec);
  (void)hipFree(mg.rec.flags);
  (void)hipFree(mg.tmpA);
  (void)hipFree(mg.tmpB);
  (void)hipFree(mg.red);
  (void)hipFree(mg.ebe);
  (void)hipFree(mg.stencil);
  (void)hipFree(mg.ebuf32);
  (void)hipFree(mg.rec64);
  (void)hipFree(mg.u64);
  mg = MGState();
}

// ---------------------------------------------------------------------------
// Linearisation: FP64 decisions -> FP32 record (one launch over all bricks).
// ---------------------------------------------------------------------------

// MODE 0: linearisation record; MODE 1: state commit into state_out.
// Records of a point with extra branches in parallel: layer 0 is the block's record,
// whose flags carry the point's history switch and whose dL slot its dL/dphi (both
// from the total psi^+); layer 1 + j that of extra branch j, or flags REC_EMPTY where
// the point's phase has no branch in slot j. Layer l of a record array sits at
// rec + l * REC_N * n_q and flags + l * n_q.
constexpr uint8_t REC_EMPTY = 0x80;

struct LinArgs {
  MeshDev m;
  int nx1, ny1;
  int64_t n_nodes, n_q;
  const double* z;
  const double* phin;
  const double* state;
  const uint8_t* phase;
  const MatParams<double>* mats;
  int nph;
  FracParams<double> fr;
  RecordSoA rec;
  double* rec64;         // MODE 0: the same record in FP64 [REC_N][n_q] (flags shared), or null
  double* state_out;
  int* flag;
  const XBranch* xb;     // extra branches [nph][n_extra] and their states [7*n_extra][n_q]
  const double* xstate;
  int n_extra;
  double* xstate_out;    // MODE 3: the extra branches' committed states
  const double* qd;      // GEO: mapped elements' geometry record [10][n_q] (J^-1, w det J)
};

// MODE 0: record; MODE 2: record with the extra branches' layers; MODE 1: state commit;
// MODE 3: state commit with the extra branches. GEO: mapped elements (gradients through
// each point's J^-1 from a.qd).
template <int P, int Q, int MODE, bool GEO = false>
__global__ __launch_bounds__(NT) void k_linearize(LinArgs a, int colour, DevTables* __restrict__ tabs) {
  using S = OpShape<P, Q>;
  constexpr int NB3 = S::NB3, Q3 = S::Q3, ER = S::ER;
  extern __shared__ double lds[];
  double* zb = lds;
  double* tmp = zb + 4 * NB3;
  double* tab = tmp + S::TMP;
  const int brick = xcd_brick(a.m, colour, blockIdx.x);
  if (brick < 0) return;  // padding workgroup (uniform)
  const BrickGeom g = decode_brick(a.m, colour, brick);
  for (int t = threadIdx.x; t < Q * P; t += NT) {
    tab[t] = tabs->B[P][Q][t / P][t % P];
    tab[Q * P + t] = tabs->D[P][Q][t / P][t % P];
  }
  stage_brick<double, double, P, 4>(a.z, a.n_nodes, a.nx1, a.ny1, g, zb);
  __syncthreads();
  const TabRef<double> tb{tab, tab + Q * P};
  const double ih[3] = {a.m.ih[0], a.m.ih[1], a.m.ih[2]};
  double* xb = tmp;
  double* xd = xb + ER * P * P * Q;
  double* ybb = xd + ER * P * P * Q;
  double* ydb = ybb + ER * P * Q * Q;
  double* ybd = ydb + ER * P * Q * Q;
  const int t = threadIdx.x;
  const int el = t / Q3, ql = t % Q3;
  const int qx = ql % Q, qy = (ql / Q) % Q, qz = ql / (Q * Q);
  bool any_bad = false, bad_pid = false;
  for (int r = 0; r < S::ROUNDS; ++r) {
    const int slot0 = r * ER, slot = slot0 + el;
    const int sx = slot & 1, sy = (slot >> 1) & 1, sz = slot >> 2;
    const bool active = (t < ER * Q3) && (slot < 8) && sx < g.nex && sy < g.ney && sz < g.nez;
    double G[9], phi = 0.0;
#pragma unroll 1
    for (int f = 0; f < 4; ++f) {
      fwd_xy<double, P, Q, ER>(zb + f * NB3, slot0, g, tb, f < 3, xb, xd, ybb, ydb, ybd);
      if (t < ER * Q3) {
        double v, d[3];
        fwd_z<double, P, Q>(ybb, ydb, ybd, el, qx, qy, qz, tb, f < 3, v, d);
        if (f < 3) {
#pragma unroll
          for (int J = 0; J < 3; ++J) G[3 * f + J] = GEO ? d[J] : d[J] * ih[J];  // GEO: mapped below
        } else {
          phi = v;
        }
      }
      __syncthreads();
    }
    if (active) {
      const int64_t e = (int64_t)(g.ex0 + sx) + (int64_t)a.m.nx * ((g.ey0 + sy) + (int64_t)a.m.ny * (g.ez0 + sz));
      const int64_t gq = e * Q3 + ql;
      if (GEO) {
        double gA[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) gA[k] = a.qd[k * a.n_q + gq];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
          const double dr[3] = {G[3 * f], G[3 * f + 1], G[3 * f + 2]};
          ref_to_phys<true>(dr, ih, gA, G + 3 * f);
        }
      }
      double st[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) st[k] = a.state[k * a.n_q + gq];
      const int pid = a.phase[gq];
      bad_pid |= pid >= a.nph;  // an id outside the phase table raises the phase flag
      const MatParams<double> mp = a.mats[pid < a.nph ? pid : 0];
      QPState<double> s;
      qp_state<double>(mp, a.fr, G, phi, 0.0, st, s);
      any_bad |= s.bad;
      if (MODE == 2) {
        // extra branches: one record layer each; the block's layer takes the point's
        // history switch and dL/dphi from the total psi^+
        double psi = s.psi;
        const int pidc = pid < a.nph ? pid : 0;
#pragma unroll 1
        for (int j = 0; j < a.n_extra; ++j) {
          const int64_t lj = 1 + j;
          const XBranch& b = a.xb[pidc * a.n_extra + j];
          if (b.kind == XB_NONE) {
            a.rec.flags[lj * a.n_q + gq] = REC_EMPTY;
            continue;
          }
          double xs[8];
#pragma unroll
          for (int k = 0; k < 7; ++k) xs[k] = b.kind == XB_HOOKE ? 0.0 : a.xstate[(int64_t)(7 * j + k) * a.n_q + gq];
          xs[7] = 0.0;
          QPState<double> sj;
          qp_state<double, true, true>(b.m, a.fr, G, phi, 0.0, xs, sj);
          any_bad |= sj.bad;
          psi += sj.psi;
          LinRecord rj;
          record_from_state(sj, rj);
#pragma unroll
          for (int k = 0; k < REC_N; ++k) a.rec.rec[(lj * REC_N + k) * a.n_q + gq] = rj.v[k];
          a.rec.flags[lj * a.n_q + gq] = rj.flags;
          if (a.rec64) {
            LinRecordT<double> r64;
            record_from_state(sj, r64);
#pragma unroll
            for (int k = 0; k < REC_N; ++k) a.rec64[(lj * REC_N + k) * a.n_q + gq] = r64.v[k];
          }
        }
        s.hactive = psi > st[7];
        const double H = s.hactive ? psi : st[7];
        const double alpha_pp = (a.fr.at == 2) ? 2.0 : 0.0;
        s.dLcoef = 2.0 * H + mp.Gc * a.fr.inv_c0l0 * alpha_pp + a.fr.zeta * a.fr.inv_dt;
      }
      if (MODE == 3) {
        // every branch's state (Box 1 step 4); the block's history takes the total psi^+
        double psi = s.psi;
        const int pidc = pid < a.nph ? pid : 0;
#pragma unroll 1
        for (int j = 0; j < a.n_extra; ++j) {
          const XBranch& b = a.xb[pidc * a.n_extra + j];
          double xs[8];
#pragma unroll
          for (int k = 0; k < 7; ++k) xs[k] = a.xstate[(int64_t)(7 * j + k) * a.n_q + gq];
          xs[7] = 0.0;
          if (b.kind == XB_NONE) {
#pragma unroll
            for (int k = 0; k < 7; ++k) a.xstate_out[(int64_t)(7 * j + k) * a.n_q + gq] = xs[k];
            continue;
          }
          double xk[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) xk[k] = b.kind == XB_HOOKE ? 0.0 : xs[k];
          QPState<double> sj;
          qp_state<double, true, true>(b.m, a.fr, G, phi, 0.0, xk, sj);
          any_bad |= sj.bad;
          psi += sj.psi;
          double nj[8];
          if (b.kind == XB_HOOKE) {
#pragma unroll
            for (int k = 0; k < 7; ++k) nj[k] = xs[k];
          } else {
            commit_from_state(sj, G, xk, nj);
          }
#pragma unroll
          for (int k = 0; k < 7; ++k) a.xstate_out[(int64_t)(7 * j + k) * a.n_q + gq] = nj[k];
        }
        s.hactive = psi > st[7];
        s.H = s.hactive ? psi : st[7];
      }
      if (MODE == 0 || MODE == 2) {
        LinRecord rc;
        record_from_state(s, rc);
#pragma unroll
        for (int k = 0; k < REC_N; ++k) a.rec.rec[k * a.n_q + gq] = rc.v[k];
        a.rec.flags[gq] = rc.flags;
        if (a.rec64) {
          LinRecordT<double> r64;
          record_from_state(s, r64);
#pragma unroll
          for (int k = 0; k < REC_N; ++k) a.rec64[k * a.n_q + gq] = r64.v[k];
        }
      } else {
        double ns[8];
        commit_from_state(s, G, st, ns);
#pragma unroll
        for (int k = 0; k < 8; ++k) a.state_out[k * a.n_q + gq] = ns[k];
      }
    }
  }
  if (any_bad) a.flag[0] = 1;
  if (bad_pid) a.flag[1] = 1;
}

// ---------------------------------------------------------------------------
// FP32 level apply (MODE 0) and point-Jacobi diagonal (MODE 1).
// PF: fine nodes per direction (kinematics), PC: this level's nodes per direction.
// ---------------------------------------------------------------------------

// Arguments of the linearised applies from a record: V = float for the FP32 multigrid
// levels, V = double for the FP64 apply from the stored linearisation (fine level).
template <typename V> struct LinApplyArgs {
  MeshDev m;
  LevelDev fine, lev;
  int64_t n_q;
  const V* z32;          // fine u at the linearisation point [3][n_fine]
  const V* dz;           // level vector [4][n_lev]
  RecordSoAT<V> rec;
  const uint8_t* phase;
  const MatParams<V>* mats;
  int nph;
  FracParams<V> fr;
  V* out;
  V* ebuf;               // brick-buffer scatter (extended node grid)
  const MatParams<V>* xmats;  // extra branches [nph][n_extra] (record layers 1..n_extra)
  int n_extra;
  const V* qd;           // GEO: mapped elements' geometry record [10][n_q] (J^-1, w det J),
                         // in the working precision
};

// Mapped elements in the record applies: reference derivatives (FP64) to a physical
// gradient in the working precision through the point's J^-1 (FP64).
template <typename V>
__device__ inline void map_grad(double d0, double d1, double d2, const double* A, V* out) {
#pragma unroll
  for (int J = 0; J < 3; ++J) out[J] = (V)(d0 * A[J] + d1 * A[3 + J] + d2 * A[6 + J]);
}

// Record-based tangent of one point: the block's layer, plus (n_extra > 0) the extra
// branches' layers, their dP and dpsi^+ summed and the switch applied to the total.
// valid = false (a lane without a point) reads no layer.
// MB = false compiles the block's tangent only (kernels launched without branches).
template <typename V, bool MB>
__device__ inline void lin_tangent(const RecordSoAT<V>& rec, int64_t n_q, const MatParams<V>* xmats, int n_extra,
                                   const MatParams<V>& mp, const QPState<V>& s, int pid, int64_t gq, bool valid,
                                   const V* G, const V* dG, V dphi, V* dP, V& dL) {
  if (!MB || n_extra == 0) {
    qp_tangent<V>(mp, s, dG, dphi, dP, dL);
    return;
  }
  V dpsi;
  qp_tangent_psi<V>(mp, s, dG, dphi, dP, dpsi, true);
#pragma unroll 1
  for (int j = 0; j < n_extra; ++j) {
    const int64_t lj = 1 + j;
    const uint8_t fl = valid ? rec.flags[lj * n_q + gq] : REC_EMPTY;
    if (fl & REC_EMPTY) continue;
    LinRecordT<V> r;
#pragma unroll
    for (int k = 0; k < REC_N; ++k) r.v[k] = rec.rec[(lj * REC_N + k) * n_q + gq];
    r.flags = fl;
    const MatParams<V>& bm = xmats[pid * n_extra + j];
    QPState<V> sj;
    qp_state_lin<V>(bm, G, r, sj);
    V dPj[9], dpj;
    qp_tangent_psi<V>(bm, sj, dG, dphi, dPj, dpj, true);
#pragma unroll
    for (int k = 0; k < 9; ++k) dP[k] += dPj[k];
    dpsi += dpj;
  }
  dL = s.dLcoef * dphi + s.gp * (s.hactive ? dpsi : V(0));
}
using A32Args = LinApplyArgs<float>;

template <int PF, int PC, int Q> struct A32Shape {
  static constexpr int PM = PF > PC ? PF : PC;
  static constexpr int NBF = 2 * PF - 1, NBF3 = NBF * NBF * NBF;
  static constexpr int NBC = 2 * PC - 1, NBC3 = NBC * NBC * NBC;
  static constexpr int PC3 = PC * PC * PC, Q3 = Q * Q * Q;
  static constexpr int ER = (NT / Q3) < 8 ? (NT / Q3) : 8;
  static constexpr int ROUNDS = (8 + ER - 1) / ER;
  static constexpr int FWD = 2 * ER * PM * PM * Q + 3 * ER * PM * Q * Q;
  static constexpr int BWD = 4 * ER * Q3 + 3 * ER * PM * Q * Q + 2 * ER * PM * PM * Q;
  static constexpr int DIAG = 25 * ER * Q3;  // 22 coefficients on the box, 25 on mapped elements
  static constexpr int TMP0 = FWD > BWD ? FWD : BWD;
  static constexpr int TMP = TMP0 > DIAG ? TMP0 : DIAG;
  static constexpr int EV = 8 * 4 * PC3;
  static constexpr int TAB = 2 * Q * PF + 2 * Q * PC + Q;
  static constexpr size_t lds_floats = (size_t)3 * NBF3 + 4 * NBC3 + EV + TMP + TAB;
  static constexpr size_t lds_bytes = lds_floats * sizeof(float);
};

// GEO: mapped elements (gradients and weights from the point's geometry record).
template <int MODE, int PF, int PC, int Q, bool MB, bool GEO = false>
__global__ __launch_bounds__(NT) void k_level32(A32Args a, int colour, DevTablesF* __restrict__ tabs) {
  using S = A32Shape<PF, PC, Q>;
  constexpr int NBF3 = S::NBF3, NBC3 = S::NBC3, PC3 = S::PC3, Q3 = S::Q3, ER = S::ER, PM = S::PM;
  extern __shared__ float ldsf[];
  float* ub = ldsf;                 // [3][NBF3] fine u
  float* wb = ub + 3 * NBF3;        // [4][NBC3] level direction
  float* ev = wb + 4 * NBC3;        // [8][4][PC3]
  float* tmp = ev + S::EV;
  float* tab = tmp + S::TMP;        // Bf, Df (Q x PF), Bc, Dc (Q x PC), w (Q)
  const int brick = xcd_brick(a.m, colour, blockIdx.x);
  if (brick < 0) return;  // padding workgroup (uniform)
  const BrickGeom g = decode_brick(a.m, colour, brick);
  for (int t = threadIdx.x; t < Q * PF; t += NT) {
    tab[t] = tabs->B[PF][Q][t / PF][t % PF];
    tab[Q * PF + t] = tabs->D[PF][Q][t / PF][t % PF];
  }
  for (int t = threadIdx.x; t < Q * PC; t += NT) {
    tab[2 * Q * PF + t] = tabs->B[PC][Q][t / PC][t % PC];
    tab[2 * Q * PF + Q * PC + t] = tabs->D[PC][Q][t / PC][t % PC];
  }
  if (threadIdx.x < Q) tab[2 * Q * PF + 2 * Q * PC + threadIdx.x] = tabs->w[Q][threadIdx.x];
  stage_brick<float, float, PF, 3>(a.z32, a.fine.n_nodes, a.fine.nx1, a.fine.ny1, g, ub);
  if (MODE == 0) stage_brick<float, float, PC, 4>(a.dz, a.lev.n_nodes, a.lev.nx1, a.lev.ny1, g, wb);
  __syncthreads();
  const TabRef<float> tf{tab, tab + Q * PF};
  const TabRef<float> tc{tab + 2 * Q * PF, tab + 2 * Q * PF + Q * PC};
  const float* wq = tab + 2 * Q * PF + 2 * Q * PC;
  const float ih[3] = {(float)a.m.ih[0], (float)a.m.ih[1], (float)a.m.ih[2]};
  const float jdet = (float)a.m.jdet;
  float* xb = tmp;
  float* xd = xb + ER * PM * PM * Q;
  float* ybb = xd + ER * PM * PM * Q;
  float* ydb = ybb + ER * PM * Q * Q;
  float* ybd = ydb + ER * PM * Q * Q;
  float* q0 = tmp;
  float* z0 = q0 + 4 * ER * Q3;
  float* zx = z0 + ER * PM * Q * Q;
  float* zy = zx + ER * PM * Q * Q;
  float* y0 = zy + ER * PM * Q * Q;
  float* yx = y0 + ER * PM * PM * Q;
  const int t = threadIdx.x;
  const int el = t / Q3, ql = t % Q3;
  const int qx = ql % Q, qy = (ql / Q) % Q, qz = ql / (Q * Q);
  for (int r = 0; r < S::ROUNDS; ++r) {
    const int slot0 = r * ER, slot = slot0 + el;
    const int sx = slot & 1, sy = (slot >> 1) & 1, sz = slot >> 2;
    const bool active = (t < ER * Q3) && (slot < 8) && sx < g.nex && sy < g.ney && sz < g.nez;
    // mapped elements: the point's J^-1 (FP64) and weight
    double gA[GEO ? 9 : 1];
    float wgeo = 0.f;
    if (GEO) {
      const int64_t e = (int64_t)(g.ex0 + sx) + (int64_t)a.m.nx * ((g.ey0 + sy) + (int64_t)a.m.ny * (g.ez0 + sz));
      const int64_t gq = e * Q3 + ql;
#pragma unroll
      for (int k = 0; k < 9; ++k) gA[k] = active ? a.qd[k * a.n_q + gq] : 0.0;
      wgeo = active ? (float)a.qd[9 * a.n_q + gq] : 0.f;
    }
    float G[9], W[9], wphi = 0.f, gw[3] = {0.f, 0.f, 0.f};
#pragma unroll 1
    for (int f = 0; f < 3; ++f) {
      fwd_xy<float, PF, Q, ER>(ub + f * NBF3, slot0, g, tf, true, xb, xd, ybb, ydb, ybd);
      if (t < ER * Q3) {
        float v, d[3];
        fwd_z<float, PF, Q>(ybb, ydb, ybd, el, qx, qy, qz, tf, true, v, d);
        if (GEO)
          map_grad<float>(d[0], d[1], d[2], gA, G + 3 * f);
        else
#pragma unroll
          for (int J = 0; J < 3; ++J) G[3 * f + J] = d[J] * ih[J];
      }
      __syncthreads();
    }
    if (MODE == 0) {
#pragma unroll 1
      for (int f = 0; f < 4; ++f) {
        fwd_xy<float, PC, Q, ER>(wb + f * NBC3, slot0, g, tc, true, xb, xd, ybb, ydb, ybd);
        if (t < ER * Q3) {
          float v, d[3];
          fwd_z<float, PC, Q>(ybb, ydb, ybd, el, qx, qy, qz, tc, true, v, d);
          float m[3];
          if (GEO)
            map_grad<float>(d[0], d[1], d[2], gA, m);
          else
#pragma unroll
            for (int J = 0; J < 3; ++J) m[J] = d[J] * ih[J];
          if (f < 3) {
#pragma unroll
            for (int J = 0; J < 3; ++J) W[3 * f + J] = m[J];
          } else {
            wphi = v;
#pragma unroll
            for (int J = 0; J < 3; ++J) gw[J] = m[J];
          }
        }
        __syncthreads();
      }
    }
    float Fu[9], f0 = 0.f, f1[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 9; ++k) Fu[k] = 0.f;
    QPState<float> s;
    MatParams<float> mp;
    float wdet = 0.f;
    int pidc = 0;
    int64_t gqa = 0;
    if (active) {
      const int64_t e = (int64_t)(g.ex0 + sx) + (int64_t)a.m.nx * ((g.ey0 + sy) + (int64_t)a.m.ny * (g.ez0 + sz));
      const int64_t gq = e * Q3 + ql;
      LinRecord rc;
#pragma unroll
      for (int k = 0; k < REC_N; ++k) rc.v[k] = a.rec.rec[k * a.n_q + gq];
      rc.flags = a.rec.flags[gq];
      const int pid = a.phase[gq];
      pidc = pid < a.nph ? pid : 0;
      gqa = gq;
      mp = a.mats[pidc];
      qp_state_lin<float>(mp, G, rc, s);
      wdet = GEO ? wgeo : wq[qx] * wq[qy] * wq[qz] * jdet;
      if (MODE == 0) {
        float dL;
        lin_tangent<float, MB>(a.rec, a.n_q, a.xmats, a.n_extra, mp, s, pidc, gq, true, G, W, wphi, Fu, dL);
#pragma unroll
        for (int k = 0; k < 9; ++k) Fu[k] *= wdet;
        f0 = wdet * a.fr.s_phi * dL;
        const float kfg = a.fr.kf * mp.Gc;
#pragma unroll
        for (int J = 0; J < 3; ++J) f1[J] = wdet * kfg * gw[J];
      }
    }
    if (MODE == 0) {
#pragma unroll 1
      for (int f = 0; f < 4; ++f) {
        if (t < ER * Q3) {
          float fl[3];
          if (f < 3) {
            q0[t] = 0.f;
#pragma unroll
            for (int J = 0; J < 3; ++J) fl[J] = Fu[3 * f + J];
          } else {
            q0[t] = f0;
#pragma unroll
            for (int J = 0; J < 3; ++J) fl[J] = f1[J];
          }
#pragma unroll
          for (int K = 0; K < 3; ++K)
            q0[(1 + K) * ER * Q3 + t] =
                GEO ? (float)(fl[0] * gA[3 * K] + fl[1] * gA[3 * K + 1] + fl[2] * gA[3 * K + 2]) : fl[K] * ih[K];
        }
        __syncthreads();
        bwd_field<float, PC, Q, ER>(q0, q0 + ER * Q3, q0 + 2 * ER * Q3, q0 + 3 * ER * Q3, f == 3, slot0, ER, tc,
                                    z0, zx, zy, y0, yx, ev, 4, f);
      }
    } else {
      // diagonal: quadratic-form coefficients per point in reference coordinates,
      // then every (element, node) pair sums over the points with the 1-D tables
      constexpr int NCF = GEO ? 25 : 22;
      float* cf = tmp;  // [NCF][ER*Q3]
      if (t < ER * Q3) {
        float c22[NCF];
#pragma unroll
        for (int k = 0; k < NCF; ++k) c22[k] = 0.f;
        if (active) {
#pragma unroll 1
          for (int i = 0; i < 3; ++i) {
            float C[3][3];
#pragma unroll 1
            for (int K = 0; K < 3; ++K) {
              float dG[9], dP[9], dL;
#pragma unroll
              for (int k = 0; k < 9; ++k) dG[k] = 0.f;
              dG[3 * i + K] = 1.f;
              lin_tangent<float, MB>(a.rec, a.n_q, a.xmats, a.n_extra, mp, s, pidc, gqa, true, G, dG, 0.f, dP, dL);
#pragma unroll
              for (int J = 0; J < 3; ++J) C[J][K] = dP[3 * i + J];
            }
            // in reference coordinates, Ch = A C A^T (A = J^-1; the box: A = diag(ih));
            // xx, yy, zz, xy, xz, yz
            float Ch[3][3];
#pragma unroll
            for (int K = 0; K < 3; ++K)
#pragma unroll
              for (int L = 0; L < 3; ++L) {
                if (GEO) {
                  double acc = 0.0;
#pragma unroll
                  for (int J = 0; J < 3; ++J)
#pragma unroll
                    for (int J2 = 0; J2 < 3; ++J2) acc += gA[3 * K + J] * (double)C[J][J2] * gA[3 * L + J2];
                  Ch[K][L] = (float)acc;
                } else {
                  Ch[K][L] = ih[K] * ih[L] * C[K][L];
                }
              }
            c22[6 * i + 0] = wdet * Ch[0][0];
            c22[6 * i + 1] = wdet * Ch[1][1];
            c22[6 * i + 2] = wdet * Ch[2][2];
            c22[6 * i + 3] = wdet * (Ch[0][1] + Ch[1][0]);
            c22[6 * i + 4] = wdet * (Ch[0][2] + Ch[2][0]);
            c22[6 * i + 5] = wdet * (Ch[1][2] + Ch[2][1]);
          }
          float dG[9], dP[9], dL;
#pragma unroll
          for (int k = 0; k < 9; ++k) dG[k] = 0.f;
          lin_tangent<float, MB>(a.rec, a.n_q, a.xmats, a.n_extra, mp, s, pidc, gqa, true, G, dG, 1.f, dP, dL);
          c22[18] = wdet * a.fr.s_phi * dL;
          const float kfg = wdet * a.fr.kf * mp.Gc;
          if (GEO) {
            // kfg A A^T: diagonal in 19..21, xy, xz, yz (doubled) in 22..24
            double M[3][3];
#pragma unroll
            for (int K = 0; K < 3; ++K)
#pragma unroll
              for (int L = 0; L < 3; ++L) M[K][L] = gA[3 * K] * gA[3 * L] + gA[3 * K + 1] * gA[3 * L + 1] + gA[3 * K + 2] * gA[3 * L + 2];
            c22[19] = kfg * (float)M[0][0];
            c22[20] = kfg * (float)M[1][1];
            c22[21] = kfg * (float)M[2][2];
            c22[NCF - 3] = kfg * (float)(2.0 * M[0][1]);
            c22[NCF - 2] = kfg * (float)(2.0 * M[0][2]);
            c22[NCF - 1] = kfg * (float)(2.0 * M[1][2]);
          } else {
            c22[19] = kfg * ih[0] * ih[0];
            c22[20] = kfg * ih[1] * ih[1];
            c22[21] = kfg * ih[2] * ih[2];
          }
        }
#pragma unroll
        for (int k = 0; k < NCF; ++k) cf[k * ER * Q3 + t] = c22[k];
      }
      __syncthreads();
      for (int o = t; o < ER * PC3; o += NT) {
        const int e2 = o / PC3, a2 = o % PC3;
        const int ax = a2 % PC, ay = (a2 / PC) % PC, az = a2 / (PC * PC);
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        for (int q = 0; q < Q3; ++q) {
          const int px = q % Q, py = (q / Q) % Q, pz = q / (Q * Q);
          const float bx = tc.B[px * PC + ax], dx = tc.D[px * PC + ax];
          const float by = tc.B[py * PC + ay], dy = tc.D[py * PC + ay];
          const float bz = tc.B[pz * PC + az], dz = tc.D[pz * PC + az];
          const float gx = dx * by * bz, gy = bx * dy * bz, gz = bx * by * dz, nn = bx * by * bz;
          const float* cq = cf + e2 * Q3 + q;
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            acc[i] += gx * gx * cq[(6 * i + 0) * ER * Q3] + gy * gy * cq[(6 * i + 1) * ER * Q3] +
                      gz * gz * cq[(6 * i + 2) * ER * Q3] + gx * gy * cq[(6 * i + 3) * ER * Q3] +
                      gx * gz * cq[(6 * i + 4) * ER * Q3] + gy * gz * cq[(6 * i + 5) * ER * Q3];
          }
          acc[3] += nn * nn * cq[18 * ER * Q3] + gx * gx * cq[19 * ER * Q3] + gy * gy * cq[20 * ER * Q3] +
                    gz * gz * cq[21 * ER * Q3];
          if (GEO) acc[3] += gx * gy * cq[(NCF - 3) * ER * Q3] + gx * gz * cq[(NCF - 2) * ER * Q3] +
                             gy * gz * cq[(NCF - 1) * ER * Q3];
        }
#pragma unroll
        for (int f = 0; f < 4; ++f) ev[((slot0 + e2) * 4 + f) * PC3 + a2] = acc[f];
      }
      __syncthreads();
    }
  }
  scatter_brick<float, PC, 4>(ev, a.m, a.lev.nx1, a.lev.ny1, a.lev.n_nodes, g, a.out);
}

// ---------------------------------------------------------------------------
// Level transfers (one direction per launch) and vector kernels.
// ---------------------------------------------------------------------------

// out[f][i2][i1][i0] = sum_k w[c*nw + k] in[f][...][base[c] + k][...] along `axis`,
// where c is the output coordinate along axis. in dims: (n0i, n1i, n2i).
static __global__ void k_transfer_1d(const float* __restrict__ in, float* __restrict__ out, int n0o, int n1o, int n2o,
                              int n0i, int n1i, int n2i, int axis, const int* __restrict__ base,
                              const float* __restrict__ w, int nw) {
  const int64_t no = (int64_t)n0o * n1o * n2o;
  const int64_t ni = (int64_t)n0i * n1i * n2i;
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < no; o += (int64_t)gridDim.x * blockDim.x) {
    const int i0 = (int)(o % n0o);
    const int i1 = (int)((o / n0o) % n1o);
    const int i2 = (int)(o / ((int64_t)n0o * n1o));
    const int c = axis == 0 ? i0 : (axis == 1 ? i1 : i2);
    const int nin = axis == 0 ? n0i : (axis == 1 ? n1i : n2i);
    const int b0 = base[c];
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    for (int k = 0; k < nw; ++k) {
      const int src = b0 + k;
      const float wk = w[(int64_t)c * nw + k];
      if (src < 0 || src >= nin || wk == 0.f) continue;
      int j0 = i0, j1 = i1, j2 = i2;
      if (axis == 0) j0 = src; else if (axis == 1) j1 = src; else j2 = src;
      const int64_t ii = j0 + (int64_t)n0i * (j1 + (int64_t)n1i * j2);
#pragma unroll
      for (int f = 0; f < 4; ++f) acc[f] += wk * in[f * ni + ii];
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) out[f * no + o] = acc[f];
  }
}

static __global__ void k_vec_zero(float* __restrict__ x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = 0.f;
}

static __global__ void k_vec_copy(const float* __restrict__ a, float* __restrict__ b, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

// y += x
static __global__ void k_vec_add(const float* __restrict__ x, float* __restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] += x[i];
}

// r = b - t
static __global__ void k_vec_sub(const float* __restrict__ b, const float* __restrict__ t, float* __restrict__ r, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    r[i] = b[i] - t[i];
}

// Chebyshev start: d = s * dinv * r ; x = (x_zero ? 0 : x) + d
static __global__ void k_cheb_first(const float* __restrict__ r, const float* __restrict__ dinv, float* __restrict__ d,
                             float* __restrict__ x, float s, int x_zero, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float di = s * dinv[i] * r[i];
    d[i] = di;
    x[i] = (x_zero ? 0.f : x[i]) + di;
  }
}

// Chebyshev step: r -= t ; d = a d + b dinv r ; x += d
static __global__ void k_cheb_step(float* __restrict__ r, const float* __restrict__ t, const float* __restrict__ dinv,
                            float* __restrict__ d, float* __restrict__ x, float a, float b, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float ri = r[i] - t[i];
    r[i] = ri;
    const float di = a * d[i] + b * dinv[i] * ri;
    d[i] = di;
    x[i] += di;
  }
}

// dinv = 1 / diag (0 where the diagonal vanishes)
static __global__ void k_vec_inv(const float* __restrict__ a, float* __restrict__ b, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i] != 0.f ? 1.f / a[i] : 0.f;
}

// x = dinv * x
static __global__ void k_vec_scale(const float* __restrict__ dinv, float* __restrict__ x, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] *= dinv[i];
}

// double-precision sum of squares, per-block partials (deterministic)
static __global__ void k_sumsq(const float* __restrict__ x, int64_t n, double* __restrict__ part) {
  __shared__ double red[NT];
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = x[i];
    s += v * v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = NT / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// b = a / ||a|| given the squared norm on the host
static __global__ void k_vec_axs(const float* __restrict__ a, float* __restrict__ b, float s, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    b[i] = s * a[i];
}

// FP64 -> FP32 mirror of the displacement rows of z
static __global__ void k_to_f32(const double* __restrict__ x, float* __restrict__ y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}

static __global__ void k_mirror_u(const double* __restrict__ z, float* __restrict__ z32, int64_t n_nodes) {
  const int64_t n = 3 * n_nodes;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    z32[i] = (float)z[i];
}

}  // namespace pfmf
