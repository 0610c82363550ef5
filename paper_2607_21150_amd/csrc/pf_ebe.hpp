// Coarsest multigrid level of order 1 as element matrices (FP32).
//
// The order-1 level operator is the Galerkin product of the fine linearised
// operator: its element matrix K_e[r][c] (r, c = field * 8 + node, 32 x 32) is the
// fine-quadrature sum of the pointwise tangent tested and tried with the order-1
// basis. It is assembled once per linearisation from the FP32 record and then
// summed into a 27-point block stencil (4 x 4 blocks per neighbour), which the
// smoother applies: the same operator as the matrix-free level apply at the fine
// quadrature, at a fraction of its cost.
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
  const MatParams<float>* xmats;  // extra branches [nph][n_extra] (record layers 1..n_extra)
  int n_extra;
  const double* qd;     // GEO: mapped elements' geometry record [10][n_q] (J^-1, w det J)
};

// One workgroup per element. The threads evaluate the tangent of the points on the
// 10 unit directions (dG_ij, dphi) into LDS; the element matrix is then the
// point sum of (test basis) x tangent x (trial basis), contracted in two steps.
// GEO: mapped elements (gradients and weights from the points' geometry record).
template <int PF, bool MB, bool GEO = false>
__global__ __launch_bounds__(NT) void k_ebe_assemble(EbeArgs a, DevTablesF* __restrict__ tabs) {
  constexpr int Q = PF, Q3 = Q * Q * Q, P3 = PF * PF * PF;
  __shared__ float ub[3 * P3];      // fine u of the element
  __shared__ float Cq[Q3][101];     // tangent columns (10 x 10) and wdet per point
  __shared__ float Bf[Q * PF], Df[Q * PF], B1[Q * 2], D1[Q * 2], wq[Q];
  constexpr int QC = 8;              // points per chunk of the second contraction
  __shared__ float Nq[Q3][8], Gq[Q3][8][3], kq[Q3];
  __shared__ float Tq[QC][10][32];
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
  // the displacement gradient of each point, once, for the NG thread groups below: one
  // task per (point, displacement field) when they fit the workgroup in one round, else
  // one per point (the basis products then serve the three fields). Gs lives in Tq, which
  // the second contraction fills only after the tangents have been taken.
  static_assert(Q3 * 9 <= QC * 10 * 32, "the point gradients fit the contraction buffer");
  float (*Gs)[9] = reinterpret_cast<float (*)[9]>(&Tq[0][0][0]);
  constexpr int NFT = 3 * Q3 <= NT ? 1 : 3;  // fields per task
  for (int task = t; task < (3 / NFT) * Q3; task += NT) {
    const int q = task % Q3, f0 = (task / Q3) * NFT;
    const int qx = q % Q, qy = (q / Q) % Q, qz = q / (Q * Q);
    float g[NFT][3];
#pragma unroll
    for (int k = 0; k < NFT; ++k) g[k][0] = g[k][1] = g[k][2] = 0.f;
    for (int n = 0; n < P3; ++n) {
      const int ax = n % PF, ay = (n / PF) % PF, az = n / (PF * PF);
      const float bx = Bf[qx * PF + ax], by = Bf[qy * PF + ay], bz = Bf[qz * PF + az];
      const float dx = Df[qx * PF + ax] * by * bz, dy = bx * Df[qy * PF + ay] * bz, dz = bx * by * Df[qz * PF + az];
#pragma unroll
      for (int k = 0; k < NFT; ++k) {
        const float u = ub[(f0 + k) * P3 + n];
        g[k][0] += u * dx;
        g[k][1] += u * dy;
        g[k][2] += u * dz;
      }
    }
    double gA[GEO ? 9 : 1];
    if (GEO) {
      const int64_t gq = e * Q3 + q;
#pragma unroll
      for (int k = 0; k < 9; ++k) gA[k] = a.qd[k * a.n_q + gq];
    }
#pragma unroll
    for (int k = 0; k < NFT; ++k) {
      if (GEO) {  // reference derivatives to physical ones
        map_grad<float>(g[k][0], g[k][1], g[k][2], gA, g[k]);
      } else {
#pragma unroll
        for (int J = 0; J < 3; ++J) g[k][J] *= ih[J];
      }
#pragma unroll
      for (int J = 0; J < 3; ++J) Gs[q][3 * (f0 + k) + J] = g[k][J];
    }
  }
  __syncthreads();
  // NG thread groups per point share its 10 tangent directions (each recomputes the point
  // state from the record)
  constexpr int NG = (NT / Q3) < 10 ? (NT / Q3) : 10;
  static_assert(NG >= 1, "a point per thread");
  if (t < NG * Q3) {
    const int q = t % Q3, grp = t / Q3;
    const int qx = q % Q, qy = (q / Q) % Q, qz = q / (Q * Q);
    float G[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) G[k] = Gs[q][k];
    const int64_t gq = e * Q3 + q;
    LinRecord rc;
#pragma unroll
    for (int k = 0; k < REC_N; ++k) rc.v[k] = a.rec.rec[k * a.n_q + gq];
    rc.flags = a.rec.flags[gq];
    const int pid = a.phase[gq];
    const int pidc = pid < a.nph ? pid : 0;
    const MatParams<float> mp = a.mats[pidc];
    QPState<float> s;
    qp_state_lin<float>(mp, G, rc, s);
    for (int in = grp; in < 10; in += NG) {
      float dG[9], dP[9], dL;
#pragma unroll
      for (int k = 0; k < 9; ++k) dG[k] = (k == in) ? 1.f : 0.f;
      lin_tangent<float, MB>(a.rec, a.n_q, a.xmats, a.n_extra, mp, s, pidc, gq, true, G, dG, in == 9 ? 1.f : 0.f, dP, dL);
#pragma unroll
      for (int o = 0; o < 9; ++o) Cq[q][o * 10 + in] = dP[o];
      Cq[q][90 + in] = dL;
    }
    if (grp == 0) Cq[q][100] = GEO ? (float)a.qd[9 * a.n_q + gq] : wq[qx] * wq[qy] * wq[qz] * jdet;
  }
  // order-1 basis at the points (values and physical gradients) and the fracture
  // gradient coefficient of each point's phase
  for (int i = t; i < Q3 * 8; i += NT) {
    const int q = i >> 3, nb = i & 7;
    const int qx = q % Q, qy = (q / Q) % Q, qz = q / (Q * Q);
    const int bx = nb & 1, by = (nb >> 1) & 1, bz = nb >> 2;
    const float vx = B1[qx * 2 + bx], vy = B1[qy * 2 + by], vz = B1[qz * 2 + bz];
    Nq[q][nb] = vx * vy * vz;
    if (GEO) {
      const int64_t gq = e * Q3 + q;
      double gA[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) gA[k] = a.qd[k * a.n_q + gq];
      float gr[3];
      map_grad<float>(D1[qx * 2 + bx] * vy * vz, vx * D1[qy * 2 + by] * vz, vx * vy * D1[qz * 2 + bz], gA, gr);
      Gq[q][nb][0] = gr[0];
      Gq[q][nb][1] = gr[1];
      Gq[q][nb][2] = gr[2];
    } else {
      Gq[q][nb][0] = D1[qx * 2 + bx] * vy * vz * ih[0];
      Gq[q][nb][1] = vx * D1[qy * 2 + by] * vz * ih[1];
      Gq[q][nb][2] = vx * vy * D1[qz * 2 + bz] * ih[2];
    }
  }
  for (int q = t; q < Q3; q += NT) {
    const int pid = a.phase[e * Q3 + q];
    kq[q] = a.fr.kf * a.mats[pid < a.nph ? pid : 0].Gc;
  }
  // Each thread owns row node na = t / 32 and column c = t % 32 (field g, node nb) for
  // the four row fields. Per chunk of points: T[q][i][c] = tangent row i applied to the
  // column's trial function, then K[f na][c] += wdet grad N_na . T[q][3f..3f+2][c]
  // (f < 3) and wdet (s_phi N_na T[q][9][c] + kf Gc grad N_na . grad N_nb [g = 3]).
  static_assert(NT == 256, "one thread per (row node, column)");
  const int na = t >> 5, c = t & 31, g = c >> 3, nbc = c & 7;
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  __syncthreads();
  for (int q0 = 0; q0 < Q3; q0 += QC) {
    const int nq = Q3 - q0 < QC ? Q3 - q0 : QC;
#pragma unroll 1
    for (int i = t; i < nq * 320; i += NT) {
      const int qq = i / 320, rem = i - qq * 320, row = rem >> 5, cc = rem & 31;
      const int gg = cc >> 3, nb = cc & 7, q = q0 + qq;
      const float* C = Cq[q];
      float v;
      if (gg < 3)
        v = C[row * 10 + 3 * gg] * Gq[q][nb][0] + C[row * 10 + 3 * gg + 1] * Gq[q][nb][1] +
            C[row * 10 + 3 * gg + 2] * Gq[q][nb][2];
      else
        v = C[row * 10 + 9] * Nq[q][nb];
      Tq[qq][row][cc] = v;
    }
    __syncthreads();
    {
#pragma unroll 2
      for (int qq = 0; qq < nq; ++qq) {
        const int q = q0 + qq;
        const float w = Cq[q][100];
        const float g0 = Gq[q][na][0], g1 = Gq[q][na][1], g2 = Gq[q][na][2];
#pragma unroll
        for (int f = 0; f < 3; ++f)
          acc[f] += w * (g0 * Tq[qq][3 * f][c] + g1 * Tq[qq][3 * f + 1][c] + g2 * Tq[qq][3 * f + 2][c]);
        float v = a.fr.s_phi * Nq[q][na] * Tq[qq][9][c];
        if (g == 3) v += kq[q] * (g0 * Gq[q][nbc][0] + g1 * Gq[q][nbc][1] + g2 * Gq[q][nbc][2]);
        acc[3] += w * v;
      }
    }
    __syncthreads();
  }
  {
#pragma unroll
    for (int f = 0; f < 4; ++f) a.K[e * 1024 + (f * 8 + na) * 32 + c] = acc[f];
  }
}

// The order-1 level as a 27-point block stencil: S[o][f][g][i] couples field f of
// node i with field g of node i + o, o = (dx + 1) + 3 (dy + 1) + 9 (dz + 1). Each
// entry sums the matching element-matrix entries over the (up to 8) elements that
// hold both nodes, in a fixed order, so the result is deterministic. One thread per
// (offset, node), nodes fastest.
static __global__ __launch_bounds__(NT) void k_stencil_from_ebe(const float* __restrict__ K, int nx, int ny, int nz,
                                                         int64_t n_nodes, float* __restrict__ S) {
  const int nx1 = nx + 1, ny1 = ny + 1;
  const int64_t n_all = 27 * n_nodes;
  for (int64_t t = blockIdx.x * (int64_t)NT + threadIdx.x; t < n_all; t += (int64_t)gridDim.x * NT) {
    const int o = (int)(t / n_nodes);
    const int64_t i = t - (int64_t)o * n_nodes;
    const int ix = (int)(i % nx1), iy = (int)((i / nx1) % ny1), iz = (int)(i / ((int64_t)nx1 * ny1));
    const int dx = o % 3 - 1, dy = (o / 3) % 3 - 1, dz = o / 9 - 1;
    float acc[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = 0.f;
#pragma unroll
    for (int na = 0; na < 8; ++na) {
      const int ax = na & 1, ay = (na >> 1) & 1, az = na >> 2;
      const int bx = ax + dx, by = ay + dy, bz = az + dz;
      const int ex = ix - ax, ey = iy - ay, ez = iz - az;
      if (bx < 0 || bx > 1 || by < 0 || by > 1 || bz < 0 || bz > 1) continue;
      if (ex < 0 || ex >= nx || ey < 0 || ey >= ny || ez < 0 || ez >= nz) continue;
      const int nb = bx + 2 * by + 4 * bz;
      const float* Ke = K + ((int64_t)ex + (int64_t)nx * (ey + (int64_t)ny * ez)) * 1024;
#pragma unroll
      for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int g = 0; g < 4; ++g) acc[4 * f + g] += Ke[(f * 8 + na) * 32 + g * 8 + nb];
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) S[((int64_t)o * 16 + k) * n_nodes + i] = acc[k];
  }
}

// Apply (MODE 0: out = S x) or diagonal (MODE 1) of the stencil; one thread per
// (node, output field), blockIdx.y = field. Reads of S are coalesced over nodes.
template <int MODE>
__global__ __launch_bounds__(NT) void k_stencil_apply(const float* __restrict__ S, int nx1, int ny1, int nz1,
                                                      int64_t n, const float* __restrict__ x,
                                                      float* __restrict__ out) {
  const int f = blockIdx.y;
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
    if (MODE == 1) {
      out[f * n + i] = S[((int64_t)13 * 16 + 5 * f) * n + i];
      continue;
    }
    const int ix = (int)(i % nx1), iy = (int)((i / nx1) % ny1), iz = (int)(i / ((int64_t)nx1 * ny1));
    float acc = 0.f;
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
      if (iz + dz < 0 || iz + dz >= nz1) continue;
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
        if (iy + dy < 0 || iy + dy >= ny1) continue;
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
          if (ix + dx < 0 || ix + dx >= nx1) continue;
          const int o = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
          const int64_t j = i + dx + (int64_t)nx1 * (dy + (int64_t)ny1 * dz);
          const float* So = S + ((int64_t)o * 16 + 4 * f) * n + i;
#pragma unroll
          for (int g = 0; g < 4; ++g) acc += So[g * n] * x[g * n + j];
        }
      }
    }
    out[f * n + i] = acc;
  }
}

// Galerkin product of a block stencil on a coarser order-1 lattice: Sc = P^T Sf P with P
// the trilinear interpolation from the coarse lattice (every second fine node per
// direction, fine n = 2 nc - 1 nodes) to the fine one; fine node 2I + a (a = -1, 0, 1)
// takes weight 1 (a = 0) or 1/2 (|a| = 1) from coarse node I. Entry (O, f, g) of coarse
// node I: sum over fine i = 2I + a and j = 2(I + O) + b with |j - i| <= 1 per direction
// of w(a) w(b) Sf[j - i][f][g][i] (accumulated in double, fixed order: deterministic).
// One thread per (offset, field pair, coarse node), nodes fastest.
static __global__ __launch_bounds__(NT) void k_stencil_rap(const float* __restrict__ Sf, int fx1, int fy1, int fz1,
                                                    float* __restrict__ Sc, int cx1, int cy1, int cz1) {
  const int64_t nf = (int64_t)fx1 * fy1 * fz1, nc = (int64_t)cx1 * cy1 * cz1;
  const int64_t n_all = 27 * 16 * nc;
  const int fd[3] = {fx1, fy1, fz1}, cd[3] = {cx1, cy1, cz1};
  for (int64_t t = blockIdx.x * (int64_t)NT + threadIdx.x; t < n_all; t += (int64_t)gridDim.x * NT) {
    const int64_t I = t % nc;
    const int rest = (int)(t / nc);
    const int k = rest % 16, O = rest / 16;
    const int Ic[3] = {(int)(I % cx1), (int)((I / cx1) % cy1), (int)(I / ((int64_t)cx1 * cy1))};
    const int dO[3] = {O % 3 - 1, (O / 3) % 3 - 1, O / 9 - 1};
    // per direction: the (fine i, offset o, weight) combinations
    int ci[3][9], co[3][9], nco[3] = {0, 0, 0};
    float cw[3][9];
    bool inside = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int J = Ic[d] + dO[d];
      if (J < 0 || J >= cd[d]) inside = false;
#pragma unroll
      for (int a = -1; a <= 1; ++a) {
        const int i = 2 * Ic[d] + a;
        if (i < 0 || i >= fd[d]) continue;
#pragma unroll
        for (int b = -1; b <= 1; ++b) {
          const int j = 2 * J + b;
          if (j < 0 || j >= fd[d] || j - i < -1 || j - i > 1) continue;
          const int m = nco[d]++;
          ci[d][m] = i;
          co[d][m] = j - i;
          cw[d][m] = (a == 0 ? 1.f : 0.5f) * (b == 0 ? 1.f : 0.5f);
        }
      }
    }
    double acc = 0.0;
    if (inside) {
      for (int mz = 0; mz < nco[2]; ++mz)
        for (int my = 0; my < nco[1]; ++my)
          for (int mx = 0; mx < nco[0]; ++mx) {
            const int on = (co[0][mx] + 1) + 3 * (co[1][my] + 1) + 9 * (co[2][mz] + 1);
            const int64_t i = ci[0][mx] + (int64_t)fx1 * (ci[1][my] + (int64_t)fy1 * ci[2][mz]);
            acc += (double)(cw[0][mx] * cw[1][my] * cw[2][mz]) * (double)Sf[((int64_t)on * 16 + k) * nf + i];
          }
    }
    Sc[((int64_t)O * 16 + k) * nc + I] = (float)acc;
  }
}

}  // namespace pfmf
