// Mapped (curved) hexahedra: the isoparametric map of Section 4, x(xi) = sum_a X_a N_a(xi),
// with node positions X given per global node. The operator kernels read a per-point
// geometry record instead of the box's constant 2/h factors:
//
//   qd[k * n_q + gq], k = 3 K + J (K, J = 0..2): (J^-1)_KJ = d xi_K / d x_J
//   qd[9 * n_q + gq]:                            w_x w_y w_z det J
//
// so a physical gradient is sum_K (d/d xi_K) (J^-1)_KJ and the transposed map of the
// backward pass is sum_J F_J (J^-1)_KJ. Points are ordered as the state
// (gq = e Q^3 + qx + Q qy + Q^2 qz), 80 bytes per point.
#pragma once
#include "pf_brick.hpp"

namespace pfmf {

constexpr int GEO_N = 10;

// One thread per point: J_iK = sum_a X_i(a) dN_a/dxi_K from the element's P^3 nodes,
// its inverse and determinant; flag[0] = 1 where det J <= 0 (an inverted element).
template <int P, int Q>
__global__ __launch_bounds__(NT) void k_geometry(const double* __restrict__ X, int64_t n_nodes, int nx1, int ny1,
                                                 int nx, int ny, int64_t n_q, const DevTables* __restrict__ tabs,
                                                 double* __restrict__ qd, int* __restrict__ flag) {
  const int64_t gq = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (gq >= n_q) return;
  constexpr int Q3 = Q * Q * Q, p = P - 1;
  const int64_t e = gq / Q3;
  const int ql = (int)(gq - e * Q3);
  const int qx = ql % Q, qy = (ql / Q) % Q, qz = ql / (Q * Q);
  const int64_t ex = e % nx, ey = (e / nx) % ny, ez = e / ((int64_t)nx * ny);
  double J[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
  for (int az = 0; az < P; ++az) {
    const double bz = tabs->B[P][Q][qz][az], dz = tabs->D[P][Q][qz][az];
    for (int ay = 0; ay < P; ++ay) {
      const double by = tabs->B[P][Q][qy][ay], dy = tabs->D[P][Q][qy][ay];
      const int64_t row = ex * p + (int64_t)nx1 * ((ey * p + ay) + (int64_t)ny1 * (ez * p + az));
      for (int ax = 0; ax < P; ++ax) {
        const double bx = tabs->B[P][Q][qx][ax], dx = tabs->D[P][Q][qx][ax];
        const double dr[3] = {dx * by * bz, bx * dy * bz, bx * by * dz};
        const int64_t node = row + ax;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const double xi = X[i * n_nodes + node];
#pragma unroll
          for (int K = 0; K < 3; ++K) J[i][K] += xi * dr[K];
        }
      }
    }
  }
  // inverse by cofactors: (J^-1)_Ki = cof(J)_iK / det J
  const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
  if (!(det > 0.0)) flag[0] = 1;
  const double id = 1.0 / det;
  double inv[3][3];
  inv[0][0] = c00 * id;
  inv[1][0] = c01 * id;
  inv[2][0] = c02 * id;
  inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
  inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
  inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
  inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
  inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
  inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
#pragma unroll
  for (int K = 0; K < 3; ++K)
#pragma unroll
    for (int Jc = 0; Jc < 3; ++Jc) qd[(3 * K + Jc) * n_q + gq] = inv[K][Jc];
  qd[9 * n_q + gq] = tabs->w[Q][qx] * tabs->w[Q][qy] * tabs->w[Q][qz] * det;
}

// The same geometry record for a table restriction: element e's local node a is global
// node conn[e P^3 + a].
template <int P, int Q>
__global__ __launch_bounds__(NT) void k_geometry_tab(const double* __restrict__ X, int64_t n_nodes,
                                                     const int32_t* __restrict__ conn, int64_t n_q,
                                                     const DevTables* __restrict__ tabs, double* __restrict__ qd,
                                                     int* __restrict__ flag) {
  const int64_t gq = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (gq >= n_q) return;
  constexpr int Q3 = Q * Q * Q, P3 = P * P * P;
  const int64_t e = gq / Q3;
  const int ql = (int)(gq - e * Q3);
  const int qx = ql % Q, qy = (ql / Q) % Q, qz = ql / (Q * Q);
  const int32_t* en = conn + e * P3;
  double J[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
  for (int az = 0; az < P; ++az) {
    const double bz = tabs->B[P][Q][qz][az], dz = tabs->D[P][Q][qz][az];
    for (int ay = 0; ay < P; ++ay) {
      const double by = tabs->B[P][Q][qy][ay], dy = tabs->D[P][Q][qy][ay];
      for (int ax = 0; ax < P; ++ax) {
        const double bx = tabs->B[P][Q][qx][ax], dx = tabs->D[P][Q][qx][ax];
        const double dr[3] = {dx * by * bz, bx * dy * bz, bx * by * dz};
        const int64_t node = en[ax + P * (ay + P * az)];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          const double xi = X[i * n_nodes + node];
#pragma unroll
          for (int K = 0; K < 3; ++K) J[i][K] += xi * dr[K];
        }
      }
    }
  }
  const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
  if (!(det > 0.0)) flag[0] = 1;
  const double id = 1.0 / det;
  double inv[3][3];
  inv[0][0] = c00 * id;
  inv[1][0] = c01 * id;
  inv[2][0] = c02 * id;
  inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
  inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
  inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
  inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
  inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
  inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
#pragma unroll
  for (int K = 0; K < 3; ++K)
#pragma unroll
    for (int Jc = 0; Jc < 3; ++Jc) qd[(3 * K + Jc) * n_q + gq] = inv[K][Jc];
  qd[9 * n_q + gq] = tabs->w[Q][qx] * tabs->w[Q][qy] * tabs->w[Q][qz] * det;
}

// Transpose of the table restriction (E^T P^T of Section 4) as a node-owner gather: node i
// sums the element-vector entries listed for it in a CSR map, ent[off[i] .. off[i+1]), each
// entry (e P3 + a) 4 (element e, local node a; the 4 fields are contiguous, so one entry is
// one 32-byte read), in the map's fixed order (by element, then local node):
// deterministic, no atomics. One thread per node.
static __global__ __launch_bounds__(NT) void k_gather_csr(const double* __restrict__ evec, const int32_t* __restrict__ off,
                                                   const int32_t* __restrict__ ent, int64_t n_nodes,
                                                   double* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)NT + threadIdx.x; i < n_nodes; i += (int64_t)gridDim.x * NT) {
    const int k0 = off[i], k1 = off[i + 1];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = k0; k < k1; ++k) {
      const double4 v = *reinterpret_cast<const double4*>(evec + ent[k]);
      acc[0] += v.x;
      acc[1] += v.y;
      acc[2] += v.z;
      acc[3] += v.w;
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) out[f * n_nodes + i] = acc[f];
  }
}

// Reference derivatives d[0..2] of one field to its physical gradient: the box's
// per-direction factor, or the point's J^-1.
template <bool GEO>
__device__ inline void ref_to_phys(const double d[3], const double ih[3], const double* A, double out[3]) {
#pragma unroll
  for (int J = 0; J < 3; ++J) out[J] = GEO ? d[0] * A[J] + d[1] * A[3 + J] + d[2] * A[6 + J] : d[J] * ih[J];
}

// The transpose: a flux against physical gradients to the reference directions.
template <bool GEO>
__device__ inline void phys_to_ref(const double f[3], const double ih[3], const double* A, double out[3]) {
#pragma unroll
  for (int K = 0; K < 3; ++K) out[K] = GEO ? f[0] * A[3 * K] + f[1] * A[3 * K + 1] + f[2] * A[3 * K + 2] : f[K] * ih[K];
}

}  // namespace pfmf
