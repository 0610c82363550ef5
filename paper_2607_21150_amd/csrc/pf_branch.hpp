// Branches in parallel at one quadrature point (Section 2.3, Box 1): the extra
// branches of a phase add their degraded Kirchhoff stresses to the block's and their
// psi^+ to its psi^+, and the history switch and the local phase-field residual are
// taken from the total (eq:history-field-linearization, eq:L-viscous). Each branch
// has its own state Cin^-1 (so its own principal frame) and its own Amor split; a
// Maxwell branch relaxes with the degraded modulus (eq:principal-directions-format-1).
// The FP64 operator kernels call these helpers after the block's own point state.
#pragma once
#include "pf_ops.hpp"

namespace pfmf {

// Nine values of one thread in LDS at a stride (the point's G, or its direction or
// cotangent): the branch loops read them back with volatile loads at every branch, so
// that they are not held in registers across the branch states (which otherwise spill).
struct Slot9 {
  double* p;
  int stride;
  __device__ void put(const double* v) const {
#pragma unroll
    for (int k = 0; k < 9; ++k) p[k * stride] = v[k];
  }
  __device__ void get(double* v) const {
    const volatile double* q = p;
#pragma unroll
    for (int k = 0; k < 9; ++k) v[k] = q[k * stride];
  }
};

// Point state of extra branch j of the phase (Box 1 steps 1-3 with the branch's
// material); a Hooke branch reads no state (Cin^-1 = I), and neither does a lane
// without a point (valid = false: gq may lie past the state arrays).
template <bool VOCE>
__device__ inline void xbranch_state(const OpArgs& a, const XBranch& b, int j, int64_t gq, bool valid,
                                     const double* G, double phi, QPState<double>& s) {
  double st[8];
  if (b.kind == XB_HOOKE || !valid) {
#pragma unroll
    for (int k = 0; k < 8; ++k) st[k] = 0.0;
  } else {
#pragma unroll
    for (int k = 0; k < 7; ++k) st[k] = a.xstate[(int64_t)(7 * j + k) * a.n_q + gq];
    st[7] = 0.0;
  }
  qp_state<double, VOCE, true>(b.m, a.fr, G, phi, phi, st, s);
}

// History field and the local phase-field residual and its phi-derivative at fixed
// history, from the point's total psi^+ (eq:L-viscous, eq:linearized-local-damage-residual).
__device__ inline void mb_fracture(const OpArgs& a, const MatParams<double>& m0, double phi, double phin,
                                   double Hn, double psi, double gp, bool& hact, double& L, double& dLcoef) {
  hact = psi > Hn;
  const double H = hact ? psi : Hn;
  const double alpha_p = (a.fr.at == 2) ? 2.0 * phi : 1.0;
  const double alpha_pp = (a.fr.at == 2) ? 2.0 : 0.0;
  L = gp * H + m0.Gc * a.fr.inv_c0l0 * alpha_p + a.fr.zeta * (phi - phin) * a.fr.inv_dt;
  dLcoef = 2.0 * H + m0.Gc * a.fr.inv_c0l0 * alpha_pp + a.fr.zeta * a.fr.inv_dt;
}

// Residual: P holds the block's first Piola stress on entry and the total on exit;
// returns L of the total psi^+.
template <bool VOCE>
__device__ inline double mb_residual(const OpArgs& a, const MatParams<double>& m0, int pid, int64_t gq,
                                     bool valid, Slot9 sG, double phi, double phin, double Hn, double psi0,
                                     double gp, double* P, bool& bad) {
  double psi = psi0;
#pragma unroll 1
  for (int j = 0; j < a.n_extra; ++j) {
    const XBranch& b = a.xb[pid * a.n_extra + j];
    if (b.kind == XB_NONE) continue;
    QPState<double> s;
    double G[9];
    sG.get(G);
    xbranch_state<VOCE>(a, b, j, gq, valid, G, phi, s);
    bad |= s.bad;
    double Pj[9];
    piola<double>(s, Pj);
#pragma unroll
    for (int k = 0; k < 9; ++k) P[k] += Pj[k];
    psi += s.psi;
  }
  bool hact;
  double L, dLcoef;
  mb_fracture(a, m0, phi, phin, Hn, psi, gp, hact, L, dLcoef);
  return L;
}

// Jacobian action: dP = sum of the branches' dP, dL = dLcoef dphi + g' dH with
// dH = sum of the branches' dpsi^+ when the total switch is on. Returns dL.
template <bool VOCE>
__device__ inline double mb_jacobian(const OpArgs& a, const MatParams<double>& m0, const QPState<double>& s0,
                                     int pid, int64_t gq, bool valid, Slot9 sG, double phi, double phin,
                                     double Hn, const double* W, Slot9 sW, double wphi, double* dP, bool& bad) {
  double dpsi;
  qp_tangent_psi<double>(m0, s0, W, wphi, dP, dpsi);
  double psi = s0.psi;
  const double gp = s0.gp;
#pragma unroll 1
  for (int j = 0; j < a.n_extra; ++j) {
    const XBranch& b = a.xb[pid * a.n_extra + j];
    if (b.kind == XB_NONE) continue;
    QPState<double> s;
    {
      double G[9];
      sG.get(G);
      xbranch_state<VOCE>(a, b, j, gq, valid, G, phi, s);
    }
    bad |= s.bad;
    double dPj[9], dpj, Wj[9];
    sW.get(Wj);
    qp_tangent_psi<double>(b.m, s, Wj, wphi, dPj, dpj);
#pragma unroll
    for (int k = 0; k < 9; ++k) dP[k] += dPj[k];
    dpsi += dpj;
    psi += s.psi;
  }
  bool hact;
  double L, dLcoef;
  mb_fracture(a, m0, phi, phin, Hn, psi, gp, hact, L, dLcoef);
  return dLcoef * wphi + gp * (hact ? dpsi : 0.0);
}

// psi^+ of the extra branches (the adjoint needs the total switch before the
// transposed branches).
template <bool VOCE>
__device__ inline double mb_psi_extra(const OpArgs& a, int pid, int64_t gq, bool valid, Slot9 sG,
                                      double phi, bool& bad) {
  double psi = 0.0;
#pragma unroll 1
  for (int j = 0; j < a.n_extra; ++j) {
    const XBranch& b = a.xb[pid * a.n_extra + j];
    if (b.kind == XB_NONE) continue;
    QPState<double> s;
    double G[9];
    sG.get(G);
    xbranch_state<VOCE>(a, b, j, gq, valid, G, phi, s);
    bad |= s.bad;
    psi += s.psi;
  }
  return psi;
}

// Adjoint, block part: Gb and phib of the block with the total switch; returns the
// psi^+ cotangent Hb (g' Lb when the switch is on, else 0) for the extra branches and
// the parameter partials.
__device__ inline double mb_adjoint_block(const OpArgs& a, const MatParams<double>& m0, const QPState<double>& s0,
                                          double psi_x, double phi, double phin, double Hn, const double* Pb,
                                          double Lb, double* Gb, double& phib, double* Xd) {
  bool hact;
  double L, dLcoef;
  mb_fracture(a, m0, phi, phin, Hn, s0.psi + psi_x, s0.gp, hact, L, dLcoef);
  const double Hb = hact ? s0.gp * Lb : 0.0;
  qp_tangent_T_psi<double>(m0, s0, Pb, Hb, dLcoef * Lb, Gb, phib, Xd);
  return Hb;
}

// Adjoint, extra branches: adds their transposed tangents (same Pb, Hb) to Gb, phib.
template <bool VOCE>
__device__ inline void mb_adjoint_extra(const OpArgs& a, int pid, int64_t gq, bool valid, Slot9 sG,
                                        double phi, Slot9 sPb, double Hb, double* Gb, double& phib) {
#pragma unroll 1
  for (int j = 0; j < a.n_extra; ++j) {
    const XBranch& b = a.xb[pid * a.n_extra + j];
    if (b.kind == XB_NONE) continue;
    QPState<double> s;
    {
      double G[9];
      sG.get(G);
      xbranch_state<VOCE>(a, b, j, gq, valid, G, phi, s);
    }
    double Gj[9], pj, Xj[3], Pb[9];
    sPb.get(Pb);
    qp_tangent_T_psi<double>(b.m, s, Pb, Hb, 0.0, Gj, pj, Xj);
#pragma unroll
    for (int k = 0; k < 9; ++k) Gb[k] += Gj[k];
    phib += pj;
  }
}

}  // namespace pfmf
