// Coarsest multigrid level of order 1 as element matrices (FP32).
//
// The order-1 level operator is the Galerkin product of the fine linearised
// operator: its element matrix K_e[r][c] (r, c = field * 8 + node, 32 x 32) is the
// fine-quadrature sum of the pointwise tangent tested and tried with the order-1
// basis. It is assembled once per linearisation from the FP32 record and then
// applied element by element: the same operator as the matrix-free level apply at
// the fine quadrature, at a fraction of its cost.
#pragma once
#include <hip/hip_runtime.h>

#include "pf_brick.hpp"
#include "pf_mg.hpp"
#include "pf_qf.hpp"

namespace pfmf {

struct EbeArgs {
  MeshDev m;
  LevelDev fine, lev;   // fine level (kinematics) and the order-1 level
  int64_t n_q;
  const float* z32;     // fine u mirror [3][n_fine]
  RecordSoA rec;
  const uint8_t* phase;
  const MatParams<float>* mats;
  int nph;
  FracParams<float> fr;
  float* K;             // [n_elem][32][32]
  const float* x;       // level vector (apply)
  float* out;           // level vector
};

// One workgroup per element. Threads q < Q^3 evaluate the tangent of their point on
// the 10 unit directions (dG_ij, dphi) into LDS; then every thread sums 4 entries of
// the element matrix over the points.
template <int PF>
__global__ __launch_bounds__(NT) void k_ebe_assemble(EbeArgs a, DevTablesF* __restrict__ tabs) {
  constexpr int Q = PF, Q3 = Q * Q * Q, P3 = PF * PF * PF;
  __shared__ float ub[3 * P3];      // fine u of the element
  __shared__ float Cq[Q3][101];     // tangent columns (10 x 10) and wdet per point
  __shared__ float Bf[Q * PF], Df[Q * PF], B1[Q * 2], D1[Q * 2], wq[Q];
  const int64_t e = blockIdx.x;
  const int ex = (int)(e % a.m.nx), ey = (int)((e / a.m.nx) % a.m.ny), ez = (int)(e / ((int64_t)a.m.nx * a.m.ny));
  const int t = threadIdx.x;
  for (int i = t; i < Q * PF; i += NT) {
    Bf[i] = tabs->B[PF][Q][i / PF][i % PF];
    Df[i] = tabs->D[PF][Q][i / PF][i % PF];
  }
  if (t < 2 * Q) {
    B1[t] = tabs->B[2][Q][t / 2][t % 2];
    D1[t] = tabs->D[2][Q][t / 2][t % 2];
  }
  if (t < Q) wq[t] = tabs->w[Q][t];
  constexpr int p = PF - 1;
  for (int i = t; i < 3 * P3; i += NT) {
    const int f = i / P3, n = i % P3;
    const int ax = n % PF, ay = (n / PF) % PF, az = n / (PF * PF);
    const int64_t gi = (int64_t)(ex * p + ax) + (int64_t)a.fine.nx1 * ((ey * p + ay) + (int64_t)a.fine.ny1 * (ez * p + az));
    ub[i] = a.z32[f * a.fine.n_nodes + gi];
  }
  __syncthreads();
  const float ih[3] = {(float)a.m.ih[0], (float)a.m.ih[1], (float)a.m.ih[2]};
  const float jdet = (float)a.m.jdet;
  for (int q = t; q < Q3; q += NT) {
    const int qx = q % Q, qy = (q / Q) % Q, qz = q / (Q * Q);
    float G[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) G[k] = 0.f;
    for (int n = 0; n < P3; ++n) {
      const int ax = n % PF, ay = (n / PF) % PF, az = n / (PF * PF);
      const float bx = Bf[qx * PF + ax], by = Bf[qy * PF + ay], bz = Bf[qz * PF + az];
      const float gx = Df[qx * PF + ax] * by * bz * ih[0];
      const float gy = bx * Df[qy * PF + ay] * bz * ih[1];
      const float gz = bx * by * Df[qz * PF + az] * ih[2];
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        const float u = ub[f * P3 + n];
        G[3 * f + 0] += u * gx;
        G[3 * f + 1] += u * gy;
        G[3 * f + 2] += u * gz;
      }
    }
    const int64_t gq = e * Q3 + q;
    LinRecord rc;
#pragma unroll
    for (int k = 0; k < REC_N; ++k) rc.v[k] = a.rec.rec[k * a.n_q + gq];
    rc.flags = a.rec.flags[gq];
    const int pid = a.phase[gq];
    const MatParams<float> mp = a.mats[pid < a.nph ? pid : 0];
    QPState<float> s;
    qp_state_lin<float>(mp, G, rc, s);
    for (int in = 0; in < 10; ++in) {
      float dG[9], dP[9], dL;
#pragma unroll
      for (int k = 0; k < 9; ++k) dG[k] = (k == in) ? 1.f : 0.f;
      qp_tangent<float>(mp, s, dG, in == 9 ? 1.f : 0.f, dP, dL);
#pragma unroll
      for (int o = 0; o < 9; ++o) Cq[q][o * 10 + in] = dP[o];
      Cq[q][90 + in] = dL;
    }
    Cq[q][100] = wq[qx] * wq[qy] * wq[qz] * jdet;
  }
  __syncthreads();
  for (int r0 = t; r0 < 1024; r0 += NT) {
    const int r = r0 >> 5, c = r0 & 31;
    const int f = r >> 3, na = r & 7, g = c >> 3, nb = c & 7;
    const int ax = na & 1, ay = (na >> 1) & 1, az = na >> 2;
    const int bx = nb & 1, by = (nb >> 1) & 1, bz = nb >> 2;
    float acc = 0.f;
    for (int q = 0; q < Q3; ++q) {
      const int qx = q % Q, qy = (q / Q) % Q, qz = q / (Q * Q);
      const float Na = B1[qx * 2 + ax] * B1[qy * 2 + ay] * B1[qz * 2 + az];
      const float ga[3] = {D1[qx * 2 + ax] * B1[qy * 2 + ay] * B1[qz * 2 + az] * ih[0],
                           B1[qx * 2 + ax] * D1[qy * 2 + ay] * B1[qz * 2 + az] * ih[1],
                           B1[qx * 2 + ax] * B1[qy * 2 + ay] * D1[qz * 2 + az] * ih[2]};
      const float Nb = B1[qx * 2 + bx] * B1[qy * 2 + by] * B1[qz * 2 + bz];
      const float gb[3] = {D1[qx * 2 + bx] * B1[qy * 2 + by] * B1[qz * 2 + bz] * ih[0],
                           B1[qx * 2 + bx] * D1[qy * 2 + by] * B1[qz * 2 + bz] * ih[1],
                           B1[qx * 2 + bx] * B1[qy * 2 + by] * D1[qz * 2 + bz] * ih[2]};
      const float* C = Cq[q];
      float v = 0.f;
      if (f < 3 && g < 3) {
#pragma unroll
        for (int J = 0; J < 3; ++J)
#pragma unroll
          for (int Kk = 0; Kk < 3; ++Kk) v += ga[J] * C[(3 * f + J) * 10 + 3 * g + Kk] * gb[Kk];
      } else if (f < 3) {
#pragma unroll
        for (int J = 0; J < 3; ++J) v += ga[J] * C[(3 * f + J) * 10 + 9] * Nb;
      } else if (g < 3) {
#pragma unroll
        for (int Kk = 0; Kk < 3; ++Kk) v += Na * a.fr.s_phi * C[90 + 3 * g + Kk] * gb[Kk];
      } else {
        const int64_t gq = e * Q3 + q;
        const int pid = a.phase[gq];
        const float kf = a.fr.kf * a.mats[pid < a.nph ? pid : 0].Gc;
        v = Na * a.fr.s_phi * C[99] * Nb + kf * (ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2]);
      }
      acc += C[100] * v;
    }
    a.K[e * 1024 + r0] = acc;
  }
}

// Apply (MODE 0: out = K x) or diagonal (MODE 1: out = diag K) of the order-1 level,
// brick-coloured like the other level kernels; thread = (element slot, row).
template <int MODE>
__global__ __launch_bounds__(NT) void k_ebe_apply(EbeArgs a, int colour) {
  __shared__ float xe[8][32];
  __shared__ float ev[8 * 4 * 8];
  const int brick = xcd_brick(a.m, colour, blockIdx.x);
  if (brick < 0) return;  // padding workgroup (uniform)
  const BrickGeom g = decode_brick(a.m, colour, brick);
  const int t = threadIdx.x;
  const int slot = t >> 5, r = t & 31;
  const int sx = slot & 1, sy = (slot >> 1) & 1, sz = slot >> 2;
  const bool active = sx < g.nex && sy < g.ney && sz < g.nez;
  const int64_t e = (int64_t)(g.ex0 + sx) + (int64_t)a.m.nx * ((g.ey0 + sy) + (int64_t)a.m.ny * (g.ez0 + sz));
  if (MODE == 0 && active) {
    const int f = r >> 3, n = r & 7;
    const int64_t gi = (int64_t)(g.ex0 + sx + (n & 1)) +
                       (int64_t)a.lev.nx1 * ((g.ey0 + sy + ((n >> 1) & 1)) + (int64_t)a.lev.ny1 * (g.ez0 + sz + (n >> 2)));
    xe[slot][r] = a.x[f * a.lev.n_nodes + gi];
  }
  __syncthreads();
  if (active) {
    const float* Kr = a.K + e * 1024 + r * 32;
    float acc = 0.f;
    if (MODE == 0) {
#pragma unroll 8
      for (int c = 0; c < 32; ++c) acc += Kr[c] * xe[slot][c];
    } else {
      acc = Kr[r];
    }
    ev[(slot * 4 + (r >> 3)) * 8 + (r & 7)] = acc;
  }
  __syncthreads();
  scatter_brick<float, 2, 4>(ev, a.m, a.lev.nx1, a.lev.ny1, a.lev.n_nodes, g, a.out);
}

}  // namespace pfmf
