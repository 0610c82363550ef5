// FP64 operator kernels: residual, Jacobian action and adjoint (device side).
#pragma once
#include "pf_brick.hpp"
#include "pf_qf.hpp"

namespace pfmf {

enum OpMode { M_RES = 0, M_JAC = 1, M_ADJ = 2 };

// Extra rheological branch of a phase, in parallel with its block (Section 2.3):
// kind XB_NONE (empty slot), XB_HOOKE (spring, Cin^-1 = I), XB_MAXWELL (m.am > 0) or
// XB_PRANDTL (m.plastic); m holds the branch's own spring and parameters.
enum { XB_NONE = 0, XB_HOOKE = 1, XB_MAXWELL = 2, XB_PRANDTL = 3 };
constexpr int MAX_EXTRA = 2;
struct XBranch {
  MatParams<double> m;
  int kind;
};

struct OpArgs {
  MeshDev m;
  int nx1, ny1;
  int64_t n_nodes, n_q;
  const double* z;
  const double* w;      // dz (Jacobian) or v (adjoint)
  const double* phin;
  const double* state;  // [8][n_q]
  const uint8_t* phase;
  const MatParams<double>* mats;
  int nph;
  FracParams<double> fr;
  double* out;
  double* gpart;        // adjoint: per-brick parameter partials [n_bricks][nph][3]
  int brick_base;       // global id of this colour's first brick (for gpart)
  double* ebuf;         // brick-buffer scatter: per-brick node sums [n_bricks][4][(2P-1)^3]
  int* flag;            // sticky non-physical flag (device)
  const XBranch* xb;    // extra branches [nph][n_extra] (n_extra = 0: none)
  const double* xstate; // their states [7*n_extra][n_q]: D[6], ebar_p per branch
  int n_extra;
  const double* qd;     // mapped elements: per-point geometry [10][n_q] (null: the box)
  // table restriction (pf_setup_mesh_table): element e's local node a is global node
  // conn[e * P^3 + a]; element vectors go to evec [n_elem][P^3][4], summed per node by
  // k_gather_csr; elements are taken in groups of 8 per workgroup
  const int32_t* conn;
  int64_t n_elem;
  double* evec;
  int n_groups;
};

template <int P, int Q> struct OpShape {
  static constexpr int NB = 2 * P - 1, NB3 = NB * NB * NB, P3 = P * P * P, Q3 = Q * Q * Q;
  static constexpr int ER = (NT / Q3) < 8 ? (NT / Q3) : 8;
  static constexpr int ROUNDS = (8 + ER - 1) / ER;
  static constexpr int FWD = 2 * ER * P * P * Q + 3 * ER * P * Q * Q;
  static constexpr int BWD = 4 * ER * Q3 + 3 * ER * P * Q * Q + 2 * ER * P * P * Q;
  static constexpr int TMP = FWD > BWD ? FWD : BWD;
  static constexpr int NSTAGE = 9;  // z (4) + dz/v (4) + phi_n (1)
  static constexpr int EV = 8 * 4 * P3;
  static constexpr int TAB = 2 * Q * P + Q;
  static constexpr int RED = NT;
  static constexpr size_t lds_doubles = (size_t)NSTAGE * NB3 + EV + TMP + TAB + RED;
  static constexpr size_t lds_bytes = lds_doubles * sizeof(double);
};

template <int MODE, int P, int Q>
__global__ __launch_bounds__(NT, P >= 5 ? 1 : 2) void k_op64(OpArgs a, int colour, DevTables* __restrict__ tabs) {
  using S = OpShape<P, Q>;
  constexpr int NB3 = S::NB3, P3 = S::P3, Q3 = S::Q3, ER = S::ER;
  extern __shared__ double lds[];
  double* zb = lds;                       // [4][NB3]
  double* wb = zb + 4 * NB3;              // [4][NB3]
  double* pnb = wb + 4 * NB3;             // [NB3]
  double* ev = pnb + NB3;                 // [8][4][P3]
  double* tmp = ev + S::EV;
  double* tab = tmp + S::TMP;             // B[Q*P], D[Q*P], w[Q]
  double* red = tab + S::TAB;

  const int brick = xcd_brick(a.m, colour, blockIdx.x);
  if (brick < 0) return;  // padding workgroup (uniform)
  const BrickGeom g = decode_brick(a.m, colour, brick);
  for (int t = threadIdx.x; t < Q * P; t += NT) {
    tab[t] = tabs->B[P][Q][t / P][t % P];
    tab[Q * P + t] = tabs->D[P][Q][t / P][t % P];
  }
  if (threadIdx.x < Q) tab[2 * Q * P + threadIdx.x] = tabs->w[Q][threadIdx.x];
  stage_brick<double, double, P, 4>(a.z, a.n_nodes, a.nx1, a.ny1, g, zb);
  if (MODE != M_RES) stage_brick<double, double, P, 4>(a.w, a.n_nodes, a.nx1, a.ny1, g, wb);
  if (MODE == M_RES) stage_brick<double, double, P, 1>(a.phin, a.n_nodes, a.nx1, a.ny1, g, pnb);
  __syncthreads();
  const TabRef<double> tb{tab, tab + Q * P};
  const double* wq = tab + 2 * Q * P;

  const double ih[3] = {a.m.ih[0], a.m.ih[1], a.m.ih[2]};
  const double jdet = a.m.jdet;
  double gsum[3] = {0.0, 0.0, 0.0};   // adjoint parameter partials of this thread
  int my_pid = -1;
  bool any_bad = false, bad_pid = false;

  // tmp sub-arrays
  double* xb = tmp;
  double* xd = xb + ER * P * P * Q;
  double* ybb = xd + ER * P * P * Q;
  double* ydb = ybb + ER * P * Q * Q;
  double* ybd = ydb + ER * P * Q * Q;
  double* q0 = tmp;                     // backward quadrature arrays [4][ER*Q3]
  double* z0 = q0 + 4 * ER * Q3;
  double* zx = z0 + ER * P * Q * Q;
  double* zy = zx + ER * P * Q * Q;
  double* y0 = zy + ER * P * Q * Q;
  double* yx = y0 + ER * P * P * Q;

  const int t = threadIdx.x;
  const int el = t / Q3, ql = t % Q3;
  const int qx = ql % Q, qy = (ql / Q) % Q, qz = ql / (Q * Q);

  for (int r = 0; r < S::ROUNDS; ++r) {
    const int slot0 = r * ER;
    const int slot = slot0 + el;
    const int sx = slot & 1, sy = (slot >> 1) & 1, sz = slot >> 2;
    const bool active = (t < ER * Q3) && (slot < 8) && sx < g.nex && sy < g.ney && sz < g.nez;

    // ---- forward sum factorisation: values at this thread's quadrature point
    double G[9], phi = 0.0, gphi[3] = {0, 0, 0}, phin = 0.0;
    double W[9], wphi = 0.0, gwphi[3] = {0, 0, 0};
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const bool grad = (f < 3) || MODE != M_JAC;
      fwd_xy<double, P, Q, ER>(zb + f * NB3, slot0, g, tb, grad, xb, xd, ybb, ydb, ybd);
      if (t < ER * Q3) {
        double v, d[3];
        fwd_z<double, P, Q>(ybb, ydb, ybd, el, qx, qy, qz, tb, grad, v, d);
        if (f < 3) {
#pragma unroll
          for (int J = 0; J < 3; ++J) G[3 * f + J] = d[J] * ih[J];
        } else {
          phi = v;
#pragma unroll
          for (int J = 0; J < 3; ++J) gphi[J] = d[J] * ih[J];
        }
      }
      __syncthreads();
    }
    if (MODE != M_RES) {
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        fwd_xy<double, P, Q, ER>(wb + f * NB3, slot0, g, tb, true, xb, xd, ybb, ydb, ybd);
        if (t < ER * Q3) {
          double v, d[3];
          fwd_z<double, P, Q>(ybb, ydb, ybd, el, qx, qy, qz, tb, true, v, d);
          if (f < 3) {
#pragma unroll
            for (int J = 0; J < 3; ++J) W[3 * f + J] = d[J] * ih[J];
          } else {
            wphi = v;
#pragma unroll
            for (int J = 0; J < 3; ++J) gwphi[J] = d[J] * ih[J];
          }
        }
        __syncthreads();
      }
    } else {
      fwd_xy<double, P, Q, ER>(pnb, slot0, g, tb, false, xb, xd, ybb, ydb, ybd);
      if (t < ER * Q3) {
        double v, d[3];
        fwd_z<double, P, Q>(ybb, ydb, ybd, el, qx, qy, qz, tb, false, v, d);
        phin = v;
      }
      __syncthreads();
    }

    // ---- pointwise function
    double Fu[9], f0 = 0.0, f1[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < 9; ++k) Fu[k] = 0.0;
    if (active) {
      const int64_t e = (int64_t)(g.ex0 + sx) + (int64_t)a.m.nx * ((g.ey0 + sy) + (int64_t)a.m.ny * (g.ez0 + sz));
      const int64_t gq = e * Q3 + ql;
      double st[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) st[k] = a.state[k * a.n_q + gq];
      const int pid = a.phase[gq];
      bad_pid |= pid >= a.nph;  // an id outside the phase table raises the phase flag
      const MatParams<double> mp = a.mats[pid < a.nph ? pid : 0];
      QPState<double> s;
      qp_state<double>(mp, a.fr, G, phi, phin, st, s);
      any_bad |= s.bad;
      const double wdet = wq[qx] * wq[qy] * wq[qz] * jdet;
      const double kfg = a.fr.kf * mp.Gc;
      if (MODE == M_RES) {
        piola<double>(s, Fu);
        f0 = a.fr.s_phi * s.L;
#pragma unroll
        for (int J = 0; J < 3; ++J) f1[J] = kfg * gphi[J];
#pragma unroll
        for (int k = 0; k < 9; ++k) Fu[k] *= wdet;
        f0 *= wdet;
#pragma unroll
        for (int J = 0; J < 3; ++J) f1[J] *= wdet;
      } else if (MODE == M_JAC) {
        double dL;
        qp_tangent<double>(mp, s, W, wphi, Fu, dL);
#pragma unroll
        for (int k = 0; k < 9; ++k) Fu[k] *= wdet;
        f0 = wdet * a.fr.s_phi * dL;
#pragma unroll
        for (int J = 0; J < 3; ++J) f1[J] = wdet * kfg * gwphi[J];
      } else {
        // cotangent at the point: (wdet grad v_u, wdet v_phi, wdet grad v_phi)
        double Pb[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) Pb[k] = wdet * W[k];
        const double f0b = wdet * wphi;
        const double Lb = a.fr.s_phi * f0b;
        double phib, Xd[3];
        qp_tangent_T<double>(mp, s, Pb, Lb, Fu, phib, Xd);
        f0 = phib;
#pragma unroll
        for (int J = 0; J < 3; ++J) f1[J] = kfg * wdet * gwphi[J];
        // parameter partials: Gc, sigma0, visc
        const double alpha_p = (a.fr.at == 2) ? 2.0 * phi : 1.0;
        gsum[0] = a.fr.s_phi * (alpha_p * a.fr.inv_c0l0 * f0b +
                                a.fr.kf / a.fr.s_phi * (gphi[0] * wdet * gwphi[0] + gphi[1] * wdet * gwphi[1] +
                                                        gphi[2] * wdet * gwphi[2]));
        if (s.plastic) {
          const double ee = s.e[0] * s.e[0] + s.e[1] * s.e[1] + s.e[2] * s.e[2];
          const double q = 2.0 * mp.mu * sqrt(1.5 * ee);
          const double w3q = 3.0 * mp.mu / q;
          const double xe = Xd[0] * s.e[0] + Xd[1] * s.e[1] + Xd[2] * s.e[2];
          // d(c e)_i = -w3q ddg e_i ; d tau^d_i = g 2 mu d(ce)_i ; dH = 2 mu c e.d(ce)
          const double base = s.g * 2.0 * mp.mu * xe + (s.hactive ? Lb * s.gp * 2.0 * mp.mu * s.c * ee : 0.0);
          gsum[1] = -w3q * s.ddg_s0 * base;
          gsum[2] = -w3q * s.ddg_visc * base;
        } else {
          gsum[1] = gsum[2] = 0.0;
        }
        my_pid = pid;
      }
    }
    // ---- transposed sum factorisation into the element vectors
    if (t < ER * Q3) {
      // field-major quadrature arrays reused per output field
      q0[t] = f0;
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      if (t < ER * Q3) {
        if (f < 3) {
          q0[t] = 0.0;
          q0[ER * Q3 + t] = Fu[3 * f + 0] * ih[0];
          q0[2 * ER * Q3 + t] = Fu[3 * f + 1] * ih[1];
          q0[3 * ER * Q3 + t] = Fu[3 * f + 2] * ih[2];
        } else {
          q0[t] = f0;
          q0[ER * Q3 + t] = f1[0] * ih[0];
          q0[2 * ER * Q3 + t] = f1[1] * ih[1];
          q0[3 * ER * Q3 + t] = f1[2] * ih[2];
        }
      }
      __syncthreads();
      bwd_field<double, P, Q, ER>(q0, q0 + ER * Q3, q0 + 2 * ER * Q3, q0 + 3 * ER * Q3, f == 3, slot0, ER, tb,
                                  z0, zx, zy, y0, yx, ev, 4, f);
    }
    if (MODE == M_ADJ) {
      // deterministic per-phase block reduction of the parameter partials
      for (int ph = 0; ph < a.nph; ++ph) {
        for (int k = 0; k < 3; ++k) {
          red[t] = (my_pid == ph) ? gsum[k] : 0.0;
          __syncthreads();
          for (int sstep = NT / 2; sstep > 0; sstep >>= 1) {
            if (t < sstep) red[t] += red[t + sstep];
            __syncthreads();
          }
          if (t == 0) {
            double* gp = a.gpart + ((int64_t)(a.brick_base + brick) * a.nph + ph) * 3 + k;
            *gp = (r == 0 ? 0.0 : *gp) + red[0];
          }
          __syncthreads();
        }
      }
      my_pid = -1;
    }
  }
  scatter_brick<double, P, 4>(ev, a.m, a.nx1, a.ny1, a.n_nodes, g, a.out);
  if (any_bad) a.flag[0] = 1;
  if (bad_pid) a.flag[1] = 1;
}

// flag[1] = 1 when some phase id is outside the phase table [0, nph).
static __global__ void k_check_phase(const uint8_t* __restrict__ ph, int64_t n, int nph, int* __restrict__ flag) {
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    bad |= ph[i] >= nph;
  if (bad) flag[1] = 1;
}

// Deterministic final sum of per-brick parameter partials: out[ph*3+k] = sum_b gpart[b][ph][k].
static __global__ void k_sum_params(const double* __restrict__ gpart, int n_bricks, int nph, double* __restrict__ out) {
  __shared__ double red[NT];
  const int idx = blockIdx.x;  // ph*3 + k
  double s = 0.0;
  for (int b = threadIdx.x; b < n_bricks; b += NT) s += gpart[(int64_t)b * nph * 3 + idx];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = NT / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[idx] = red[0];
}

}  // namespace pfmf
