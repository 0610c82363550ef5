// Order-4 elements (5 nodes and 5 Gauss points per direction): FP64 operator
// kernels and the FP32 multigrid level apply.
//
// One element per 128-thread workgroup. Elements are launched in 8 colours by the
// parity of their coordinates; elements of one colour share no node, and a node is
// stored by the first colour that touches it and accumulated by the later ones, so
// the scatter-add is deterministic without atomics.
//
// Sum factorisation (Section 4, B_I and B_xi) runs on up to four fields at once in
// row layout: a pass contracts one direction, and each thread owns one (field, row)
// of the element, holds the row's P inputs in registers and produces all Q outputs
// along it. Per field that is P (or Q) LDS reads per Q outputs, against P reads per
// output when each thread owns one output. The forward passes interpolate values only
// (x, y, z), and the reference gradient is then formed from the point values with the
// collocated Gauss-point derivative along x, y and z lines; the backward passes apply
// the transposes in the opposite order, ping-ponging two LDS buffers. The pointwise
// function runs with one thread per quadrature point (125 of the 128 threads). The 1-D
// tables are read with compile-time indices, so they live in scalar registers.
#pragma once
#include <hip/hip_runtime.h>

#include "pf_brick.hpp"
#include "pf_mg.hpp"
#include "pf_ops.hpp"
#include "pf_branch.hpp"
#include "pf_geom.hpp"
#include "pf_qf.hpp"
#include "pf_mfma.hpp"

namespace pfmf {

constexpr int NT5 = 128;  // threads per workgroup (one element)

// Element of colour `colour` for workgroup id (XCD-aware order as for bricks: one
// colour's elements of an x-row run on one XCD back to back); -1 for padding.
struct ElemGeom {
  int ex, ey, ez;
};
__device__ inline bool xcd_elem(const MeshDev& m, int colour, int id, ElemGeom& g) {
  const int cx = colour & 1, cy = (colour >> 1) & 1, cz = (colour >> 2) & 1;
  const int CX = (m.nx - cx + 1) / 2, CY = (m.ny - cy + 1) / 2, CZ = (m.nz - cz + 1) / 2;
  const int t = id >> 3;
  const int row = (t / CX) * 8 + (id & 7);
  if (row >= CY * CZ) return false;
  g.ex = cx + 2 * (t % CX);
  g.ey = cy + 2 * (row % CY);
  g.ez = cz + 2 * (row / CY);
  return true;
}

// All elements in one launch (element vectors): the same XCD-aware order (an x-row of
// elements on one XCD, back to back).
__host__ __device__ inline int xcd_grid_elems(int nx, int ny, int nz) { return ((ny * nz + 7) / 8) * 8 * nx; }
__device__ inline bool xcd_elem_all(const MeshDev& m, int id, ElemGeom& g) {
  const int t = id >> 3;
  const int row = (t / m.nx) * 8 + (id & 7);
  if (row >= m.ny * m.nz) return false;
  g.ex = t % m.nx;
  g.ey = row % m.ny;
  g.ez = row / m.ny;
  return true;
}

// Store the element vector R[f][k][j][i] (NF fields of P^3 nodes) into the extended node
// grid ev [NF][nz P][ny P][nx P], in which every element owns its P nodes per axis (face
// nodes appear once per element holding them); k_gather_ext<T, P> sums them per node.
// Each row of P values is contiguous, and the next element along x (launched next on the
// same XCD) writes the adjacent P values.
// Thread n < P^3 owns the element's local node n = i + P (j + P k) in every gather and
// store, so that its address is formed once for all fields.
template <typename T, int P, int NF>
__device__ inline void store_ext(const T* R, const MeshDev& m, const ElemGeom& g, T* __restrict__ ev) {
  static_assert(P * P * P <= NT5, "one thread per element node");
  constexpr int P3 = P * P * P;
  const int n = threadIdx.x;
  if (n >= P3) return;
  const int64_t NXe = (int64_t)m.nx * P, NYe = (int64_t)m.ny * P, NZe = (int64_t)m.nz * P;
  const int i = n % P, j = (n / P) % P, k = n / (P * P);
  T* d = ev + (((int64_t)g.ez * P + k) * NYe + (int64_t)g.ey * P + j) * NXe + (int64_t)g.ex * P + i;
  const int64_t fs = NZe * NYe * NXe;
#pragma unroll
  for (int f = 0; f < NF; ++f) d[f * fs] = R[f * P3 + n];
}

// Global node of local node n = i + P (j + P k) of element g on an order P-1 lattice with
// nx1 x ny1 nodes per layer.
template <int P>
__device__ inline int64_t lattice_node(int nx1, int ny1, const ElemGeom& g, int n) {
  constexpr int p = P - 1;
  const int i = n % P, j = (n / P) % P, k = n / (P * P);
  return (int64_t)(g.ex * p + i) + (int64_t)nx1 * ((g.ey * p + j) + (int64_t)ny1 * (g.ez * p + k));
}

// Global node of the thread's local node; -1 for threads beyond the P^3 nodes.
template <int P>
__device__ inline int64_t elem_node(int nx1, int ny1, const ElemGeom& g) {
  static_assert(P * P * P <= NT5, "one thread per element node");
  const int n = threadIdx.x;
  return n < P * P * P ? lattice_node<P>(nx1, ny1, g, n) : -1;
}

// Gather NF fields of the element's P^3 nodes into U[f][n]; gn = the thread's global node
// (elem_node, or the element's row of the element-to-node table for the table restriction).
template <typename T, typename S, int P, int NF>
__device__ inline void gather_nodes(const S* __restrict__ src, int64_t n_nodes, int64_t gn, T* U) {
  constexpr int P3 = P * P * P;
  const int n = threadIdx.x;
  if (n < P3) {
    T v[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) v[f] = (T)src[f * n_nodes + gn];
#pragma unroll
    for (int f = 0; f < NF; ++f) U[f * P3 + n] = v[f];
  }
}

// Table restriction: the element vector R[f][n] stored node-major, ev[(e P^3 + n) 4 + f]
// (the four fields of one entry contiguous), summed per node by k_gather_csr.
template <typename T, int P>
__device__ inline void store_elem_tab(const T* R, int64_t e, T* __restrict__ ev) {
  static_assert(P * P * P <= NT5, "one thread per element node");
  constexpr int P3 = P * P * P;
  const int n = threadIdx.x;
  if (n >= P3) return;
  T* d = ev + (e * P3 + n) * 4;
#pragma unroll
  for (int f = 0; f < 4; ++f) d[f] = R[f * P3 + n];
}

// Add the element vector R[f][k][j][i] into dst with the colour rule.
template <typename T, int P, int NF>
__device__ inline void scatter_elem(const T* R, const MeshDev& m, int nx1, int ny1, int64_t n_nodes,
                                    const ElemGeom& g, T* __restrict__ dst) {
  constexpr int p = P - 1, P3 = P * P * P;
  for (int t = threadIdx.x; t < NF * P3; t += NT5) {
    const int f = t / P3, n = t - f * P3;
    const int i = n % P, j = (n / P) % P, k = n / (P * P);
    const bool shx = (i == 0 && g.ex > 0) || (i == p && g.ex < m.nx - 1);
    const bool shy = (j == 0 && g.ey > 0) || (j == p && g.ey < m.ny - 1);
    const bool shz = (k == 0 && g.ez > 0) || (k == p && g.ez < m.nz - 1);
    const bool store = !((shx && (g.ex & 1)) || (shy && (g.ey & 1)) || (shz && (g.ez & 1)));
    const int64_t gi = (int64_t)(g.ex * p + i) + (int64_t)nx1 * ((g.ey * p + j) + (int64_t)ny1 * (g.ez * p + k));
    T* d = dst + f * n_nodes + gi;
    if (store) *d = R[t];
    else *d += R[t];
  }
}

// Slot of component c (0 value, 1..3 d/dxi_x, d/dxi_y, d/dxi_z) of field f in the point
// arrays Qo / Qi. CV (compact, four fields u_x, u_y, u_z, phi): the displacement fields
// have no value slot (the operator reads only their gradients and tests them only against
// gradients), so 13 arrays instead of 16; otherwise 4 f + c.
template <bool CV>
__device__ __forceinline__ constexpr int qslot(int f, int c) {
  return CV ? (f < 3 ? 3 * f + c - 1 : 9 + c) : 4 * f + c;
}

// Runs f(task) for task = 0 .. NTASK-1 spread over the NTH threads of the workgroup (a
// single guarded call when the workgroup has a thread per task).
template <int NTASK, int NTH, typename F>
__device__ __forceinline__ void for_tasks(F&& f) {
  if constexpr (NTASK <= NTH) {
    if ((int)threadIdx.x < NTASK) f((int)threadIdx.x);
  } else {
    for (int k = threadIdx.x; k < NTASK; k += NTH) f(k);
  }
}

// Forward: U[f][k][j][i] (P^3 per field) -> Qo[slot(f, c)][qz][qy][qx] (Q^3 per field and
// component c = value, d/dxi_x, d/dxi_y, d/dxi_z; with CV no values for f < 3). The nodal
// values are interpolated to the points by x, y and z passes (B only), and the reference
// derivatives are then taken from the point values along each line of points with the
// Gauss-point differentiation matrix G, which is exact because the interpolant has degree
// P - 1 <= Q - 1 along the line. Per (field, line) of the element a pass costs P Q (or
// Q^2) multiply-adds, against carrying value and derivative chains through every pass.
// LDS: X (in XQ) NF P^2 Q values; Y (in UY) NF Q^2 P, followed in UY by the point values
// V (NF Q^3). GR = false: values only. NE elements at once (element e's buffers at
// UY + e la and XQ + e lb), their (field, line) tasks spread over the NTH threads. Starts
// after, and ends with, a barrier.
template <typename T, typename Tab, int P, int Q, int NF, bool CV = false, bool GR = true, int NE = 1, int NTH = NT5>
__device__ __forceinline__ void sf5_fwd(T* UY, T* XQ, const Tab* __restrict__ tb, int la = 0, int lb = 0) {
  static_assert(!CV || NF == 4, "the compact layout is for the four operator fields");
  static_assert(GR || !CV, "the compact layout carries gradients");
  constexpr int P2 = P * P, P3 = P2 * P, Q2 = Q * Q, Q3 = Q2 * Q;
  constexpr int VOFF = NF * Q2 * P;  // the point values V follow Y in UY
  // x: task (f, j, k); X[f][k][j][qx]
  for_tasks<NE * NF * P2, NTH>([&](int task) {
    const int e = task / (NF * P2), t = task - e * (NF * P2);
    const T* U = UY + e * la;
    T* X = XQ + e * lb;
    const int f = t / P2, r = t - f * P2;
    T u[P];
#pragma unroll
    for (int i = 0; i < P; ++i) u[i] = U[f * P3 + r * P + i];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      T b = T(0);
#pragma unroll
      for (int i = 0; i < P; ++i) b += (T)tb->B[P][Q][q][i] * u[i];
      X[f * P2 * Q + r * Q + q] = b;
    }
  });
  __syncthreads();
  // y: task (f, qx, k); Y[f][qy][qx][k]
  for_tasks<NE * NF * Q * P, NTH>([&](int task) {
    const int e = task / (NF * Q * P), t = task - e * (NF * Q * P);
    const T* X = XQ + e * lb;
    T* Y = UY + e * la;
    const int f = t / (Q * P), s = t - f * (Q * P);
    const int qx = s % Q, k = s / Q;
    T x[P];
#pragma unroll
    for (int j = 0; j < P; ++j) x[j] = X[f * P2 * Q + (j + P * k) * Q + qx];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      T b = T(0);
#pragma unroll
      for (int j = 0; j < P; ++j) b += (T)tb->B[P][Q][q][j] * x[j];
      Y[f * Q2 * P + (qx + Q * q) * P + k] = b;
    }
  });
  __syncthreads();
  // z: task (f, qx, qy); values V[f][qz][qy][qx], and d/dxi_z along the same line
  for_tasks<NE * NF * Q2, NTH>([&](int task) {
    const int e = task / (NF * Q2), t = task - e * (NF * Q2);
    const T* Y = UY + e * la;
    T* V = UY + e * la + VOFF;
    T* O = XQ + e * lb;
    const int f = t / Q2, s = t - f * Q2;
    T y[P], v[Q];
#pragma unroll
    for (int k = 0; k < P; ++k) y[k] = Y[f * Q2 * P + s * P + k];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      T b = T(0);
#pragma unroll
      for (int k = 0; k < P; ++k) b += (T)tb->B[P][Q][q][k] * y[k];
      v[q] = b;
      const int o = s + Q2 * q;
      if (GR) V[f * Q3 + o] = b;
      if (!CV || f == 3) O[qslot<CV>(f, 0) * Q3 + o] = b;
    }
    if (GR) {
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        T d = T(0);
#pragma unroll
        for (int m = 0; m < Q; ++m) d += (T)tb->G[Q][q][m] * v[m];
        O[qslot<CV>(f, 3) * Q3 + s + Q2 * q] = d;
      }
    }
  });
  __syncthreads();
  if (!GR) return;
  // d/dxi_x along x lines: task (f, qy, qz)
  for_tasks<NE * NF * Q2, NTH>([&](int task) {
    const int e = task / (NF * Q2), t = task - e * (NF * Q2);
    const T* V = UY + e * la + VOFF;
    T* O = XQ + e * lb;
    const int f = t / Q2, s = t - f * Q2;
    T v[Q];
#pragma unroll
    for (int m = 0; m < Q; ++m) v[m] = V[f * Q3 + s * Q + m];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      T d = T(0);
#pragma unroll
      for (int m = 0; m < Q; ++m) d += (T)tb->G[Q][q][m] * v[m];
      O[qslot<CV>(f, 1) * Q3 + s * Q + q] = d;
    }
  });
  // d/dxi_y along y lines: task (f, qx, qz)
  for_tasks<NE * NF * Q2, NTH>([&](int task) {
    const int e = task / (NF * Q2), t = task - e * (NF * Q2);
    const T* V = UY + e * la + VOFF;
    T* O = XQ + e * lb;
    const int f = t / Q2, s = t - f * Q2;
    const int base = f * Q3 + (s % Q) + Q2 * (s / Q);
    T v[Q];
#pragma unroll
    for (int m = 0; m < Q; ++m) v[m] = V[base + Q * m];
    const int ob = qslot<CV>(f, 2) * Q3 + (s % Q) + Q2 * (s / Q);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      T d = T(0);
#pragma unroll
      for (int m = 0; m < Q; ++m) d += (T)tb->G[Q][q][m] * v[m];
      O[ob + Q * q] = d;
    }
  });
  __syncthreads();
}

// Transposed: Qi[slot(f, c)][q] (c = value test, tests against d/dxi_x, d/dxi_y,
// d/dxi_z; in XQ; with CV no value tests for f < 3) -> R[f][k][j][i] (in ZR). The
// derivative tests are moved back onto the point values with G^T along x, y and z lines
// and added to the value test (A[f][q] in ZR), which then goes through the transposed
// interpolation passes z, y, x. Z (in ZR, after A) holds NF P Q^2 values, Y (in XQ) NF P^2 Q.
// NE elements at once as in sf5_fwd. Starts after, and ends with, a barrier.
template <typename T, typename Tab, int P, int Q, int NF, bool CV = false, int NE = 1, int NTH = NT5>
__device__ __forceinline__ void sf5_bwd(T* XQ, T* ZR, const Tab* __restrict__ tb, int lb = 0, int la = 0) {
  static_assert(!CV || NF == 4, "the compact layout is for the four operator fields");
  constexpr int P2 = P * P, P3 = P2 * P, Q2 = Q * Q, Q3 = Q2 * Q;
  constexpr int ZOFF = NF * Q3;  // Z follows A in ZR
  // x lines: task (f, qy, qz); A = value test + G^T (x tests)
  for_tasks<NE * NF * Q2, NTH>([&](int task) {
    const int e = task / (NF * Q2), t = task - e * (NF * Q2);
    const T* I = XQ + e * lb;
    T* A = ZR + e * la;
    const int f = t / Q2, s = t - f * Q2;
    T g[Q];
#pragma unroll
    for (int m = 0; m < Q; ++m) g[m] = I[qslot<CV>(f, 1) * Q3 + s * Q + m];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      T v = (!CV || f == 3) ? I[qslot<CV>(f, 0) * Q3 + s * Q + q] : T(0);
#pragma unroll
      for (int m = 0; m < Q; ++m) v += (T)tb->G[Q][m][q] * g[m];
      A[f * Q3 + s * Q + q] = v;
    }
  });
  __syncthreads();
  // y lines: task (f, qx, qz); A += G^T (y tests)
  for_tasks<NE * NF * Q2, NTH>([&](int task) {
    const int e = task / (NF * Q2), t = task - e * (NF * Q2);
    const T* I = XQ + e * lb;
    T* A = ZR + e * la;
    const int f = t / Q2, s = t - f * Q2;
    const int o = (s % Q) + Q2 * (s / Q);
    T g[Q];
#pragma unroll
    for (int m = 0; m < Q; ++m) g[m] = I[qslot<CV>(f, 2) * Q3 + o + Q * m];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      T v = A[f * Q3 + o + Q * q];
#pragma unroll
      for (int m = 0; m < Q; ++m) v += (T)tb->G[Q][m][q] * g[m];
      A[f * Q3 + o + Q * q] = v;
    }
  });
  __syncthreads();
  // z lines: task (f, qx, qy); A + G^T (z tests), then the transposed z interpolation:
  // Z[f][k][qy][qx]
  for_tasks<NE * NF * Q2, NTH>([&](int task) {
    const int e = task / (NF * Q2), t = task - e * (NF * Q2);
    const T* I = XQ + e * lb;
    const T* A = ZR + e * la;
    T* Z = ZR + e * la + ZOFF;
    const int f = t / Q2, s = t - f * Q2;
    T g[Q], c[Q];
#pragma unroll
    for (int m = 0; m < Q; ++m) g[m] = I[qslot<CV>(f, 3) * Q3 + s + Q2 * m];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      T v = A[f * Q3 + s + Q2 * q];
#pragma unroll
      for (int m = 0; m < Q; ++m) v += (T)tb->G[Q][m][q] * g[m];
      c[q] = v;
    }
#pragma unroll
    for (int k = 0; k < P; ++k) {
      T z = T(0);
#pragma unroll
      for (int q = 0; q < Q; ++q) z += (T)tb->B[P][Q][q][k] * c[q];
      Z[f * P * Q2 + k * Q2 + s] = z;
    }
  });
  __syncthreads();
  // y^T: task (f, qx, k); Y[f][k][j][qx]
  for_tasks<NE * NF * Q * P, NTH>([&](int task) {
    const int e = task / (NF * Q * P), t = task - e * (NF * Q * P);
    const T* Z = ZR + e * la + ZOFF;
    T* Y = XQ + e * lb;
    const int f = t / (Q * P), s = t - f * (Q * P);
    const int qx = s % Q, k = s / Q;
    T v[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) v[q] = Z[f * P * Q2 + k * Q2 + q * Q + qx];
#pragma unroll
    for (int j = 0; j < P; ++j) {
      T a = T(0);
#pragma unroll
      for (int q = 0; q < Q; ++q) a += (T)tb->B[P][Q][q][j] * v[q];
      Y[f * P2 * Q + (j + P * k) * Q + qx] = a;
    }
  });
  __syncthreads();
  // x^T: task (f, j, k); R[f][k][j][i]
  for_tasks<NE * NF * P2, NTH>([&](int task) {
    const int e = task / (NF * P2), t = task - e * (NF * P2);
    const T* Y = XQ + e * lb;
    T* R = ZR + e * la;
    const int f = t / P2, r = t - f * P2;
    T y[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) y[q] = Y[f * P2 * Q + r * Q + q];
#pragma unroll
    for (int i = 0; i < P; ++i) {
      T a = T(0);
#pragma unroll
      for (int q = 0; q < Q; ++q) a += (T)tb->B[P][Q][q][i] * y[q];
      R[f * P3 + r * P + i] = a;
    }
  });
  __syncthreads();
}

// LDS sizes (values) of the two buffers for up to 4 fields (CV: the compact point arrays).
template <int P, int Q, bool CV = false> struct Q5Lds {
  static constexpr int a0 = 4 * P * P * P, a1 = 4 * Q * Q * P + 4 * Q * Q * Q;
  static constexpr int A = a0 > a1 ? a0 : a1;  // U, then Y and V (forward); A and Z, then R (backward)
  static constexpr int b0 = 4 * P * P * Q, b1 = (CV ? 13 : 16) * Q * Q * Q;
  static constexpr int B = b0 > b1 ? b0 : b1;  // X, then the point arrays (forward); point arrays, then Y (backward)
};

// FP64 residual / Jacobian / adjoint on order-4 elements.
// GEO: mapped elements (J^-1 and weight per point from a.qd). EV: all elements in one
// launch, element vectors stored to the extended node grid a.evec (summed per node by
// k_gather_ext); otherwise one colour, added into a.out by the colour rule. TAB (with
// GEO): table restriction, element e = workgroup (XCD-aware order), nodes from a.conn,
// the element vector stored node-major to a.evec (summed per node by k_gather_csr).
template <int MODE, bool VOCE, bool MB, bool GEO, bool EV = false, bool TAB = false>
__global__ __launch_bounds__(NT5, 2) void k_op64_q4(OpArgs a, int colour, DevTables* __restrict__ tabs) {
  static_assert(!TAB || (GEO && !MB), "the table restriction runs on mapped elements without branches");
  constexpr int P = 5, Q = 5, Q3 = 125;
  // compact point arrays (13 of 125 values each): 25 KB of LDS per element instead of 28,
  // so that six elements fit a CU's 160 KB (3 waves per SIMD, which the VGPRs allow)
  using L = Q5Lds<P, Q, true>;
  __shared__ double bufA[L::A];
  __shared__ double bufB[L::B];
  __shared__ double red[2 * 3 * 8];
  __shared__ double mbs[MB ? 18 * NT5 : 1];  // branches in parallel: G and W (or Pb) per thread
  const Slot9 sG{mbs + threadIdx.x, NT5}, sW{mbs + 9 * NT5 + threadIdx.x, NT5};
  ElemGeom g{0, 0, 0};
  int64_t e;
  if (TAB) {
    const int id = xcd_group(a.n_groups, blockIdx.x);
    if (id < 0) return;  // padding (uniform)
    e = id;
  } else {
    if (!(EV ? xcd_elem_all(a.m, blockIdx.x, g) : xcd_elem(a.m, colour, blockIdx.x, g))) return;  // padding (uniform)
    e = (int64_t)g.ex + (int64_t)a.m.nx * (g.ey + (int64_t)a.m.ny * g.ez);
  }
  const int t = threadIdx.x;
  // the thread's element node (every gather below reads it)
  const int64_t gn = TAB ? (t < P * P * P ? (int64_t)a.conn[e * (P * P * P) + t] : -1) : elem_node<P>(a.nx1, a.ny1, g);
  const bool pt = t < Q3;
  const int ql = pt ? t : 0;
  const int qx = ql % Q, qy = (ql / Q) % Q, qz = ql / (Q * Q);
  const int64_t gq = e * Q3 + ql;
  // per-point state, issued before the gathers
  double st[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) st[k] = pt ? a.state[k * a.n_q + gq] : 0.0;
  const int pid = pt ? a.phase[gq] : 0;
  const double ih[3] = {a.m.ih[0], a.m.ih[1], a.m.ih[2]};
  double wdet = tabs->w[Q][qx] * tabs->w[Q][qy] * tabs->w[Q][qz] * a.m.jdet;
  // mapped elements: the point's J^-1 and weight
  double gA[GEO ? 9 : 1];
  if (GEO) {
#pragma unroll
    for (int k = 0; k < 9; ++k) gA[k] = pt ? a.qd[k * a.n_q + gq] : 0.0;
    wdet = pt ? a.qd[9 * a.n_q + gq] : 0.0;
  }
  gather_nodes<double, double, P, 4>(a.z, a.n_nodes, gn, bufA);
  __syncthreads();
  sf5_fwd<double, DevTables, P, Q, 4, true>(bufA, bufB, tabs);
  double G[9], phi, gphi[3];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const double dr[3] = {bufB[qslot<true>(f, 1) * Q3 + ql], bufB[qslot<true>(f, 2) * Q3 + ql], bufB[qslot<true>(f, 3) * Q3 + ql]};
    ref_to_phys<GEO>(dr, ih, gA, f < 3 ? G + 3 * f : gphi);
  }
  phi = bufB[qslot<true>(3, 0) * Q3 + ql];
  double phin = 0.0;
  __syncthreads();
  if (MODE == M_RES) {
    gather_nodes<double, double, P, 1>(a.phin, a.n_nodes, gn, bufA);
    __syncthreads();
    sf5_fwd<double, DevTables, P, Q, 1, false, false>(bufA, bufB, tabs);
    phin = bufB[ql];
    __syncthreads();
  }
  const int pidc = pid < a.nph ? pid : 0;
  const MatParams<double> mp = a.mats[pidc];
  // branches in parallel (flags of threads without a point are dropped)
  bool xbad = false;
  double psi_x = 0.0;
  if (MB) sG.put(G);
  if (MB && MODE == M_ADJ) psi_x = mb_psi_extra<VOCE>(a, pidc, gq, pt, sG, phi, xbad);
  QPState<double> s;
  qp_state<double, VOCE>(mp, a.fr, G, phi, phin, st, s);
  bool bad = pt && s.bad;
  const bool bad_pid = pt && pid >= a.nph;  // an id outside the phase table raises the phase flag
  double W[9], wphi = 0.0, gw[3] = {0.0, 0.0, 0.0};
  if (MODE != M_RES) {
    gather_nodes<double, double, P, 4>(a.w, a.n_nodes, gn, bufA);
    __syncthreads();
    sf5_fwd<double, DevTables, P, Q, 4, true>(bufA, bufB, tabs);
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const double dr[3] = {bufB[qslot<true>(f, 1) * Q3 + ql], bufB[qslot<true>(f, 2) * Q3 + ql], bufB[qslot<true>(f, 3) * Q3 + ql]};
      ref_to_phys<GEO>(dr, ih, gA, f < 3 ? W + 3 * f : gw);
    }
    wphi = bufB[qslot<true>(3, 0) * Q3 + ql];
    __syncthreads();
  }
  const double kfg = a.fr.kf * mp.Gc;
  double Fu[9], f0, f1[3];
  double gsum[3] = {0.0, 0.0, 0.0};
  if (MODE == M_RES) {
    piola<double>(s, Fu);
    double Lr = s.L;
    if (MB) Lr = mb_residual<VOCE>(a, mp, pidc, gq, pt, sG, phi, phin, st[7], s.psi, s.gp, Fu, xbad);
#pragma unroll
    for (int k = 0; k < 9; ++k) Fu[k] *= wdet;
    f0 = wdet * a.fr.s_phi * Lr;
#pragma unroll
    for (int J = 0; J < 3; ++J) f1[J] = wdet * kfg * gphi[J];
  } else if (MODE == M_JAC) {
    double dL;
    if (MB) {
      sW.put(W);
      dL = mb_jacobian<VOCE>(a, mp, s, pidc, gq, pt, sG, phi, phi, st[7], W, sW, wphi, Fu, xbad);
    } else
      qp_tangent<double>(mp, s, W, wphi, Fu, dL);
#pragma unroll
    for (int k = 0; k < 9; ++k) Fu[k] *= wdet;
    f0 = wdet * a.fr.s_phi * dL;
#pragma unroll
    for (int J = 0; J < 3; ++J) f1[J] = wdet * kfg * gw[J];
  } else {
    double Pb[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Pb[k] = wdet * W[k];
    const double f0b = wdet * wphi;
    const double Lb = a.fr.s_phi * f0b;
    double phib, Xd[3], Hb = 0.0;
    if (MB)
      Hb = mb_adjoint_block(a, mp, s, psi_x, phi, phi, st[7], Pb, Lb, Fu, phib, Xd);
    else
      qp_tangent_T<double>(mp, s, Pb, Lb, Fu, phib, Xd);
#pragma unroll
    for (int J = 0; J < 3; ++J) f1[J] = kfg * wdet * gw[J];
    const double alpha_p = (a.fr.at == 2) ? 2.0 * phi : 1.0;
    gsum[0] = alpha_p * a.fr.inv_c0l0 * Lb + a.fr.kf * wdet * (gphi[0] * gw[0] + gphi[1] * gw[1] + gphi[2] * gw[2]);
    if (s.plastic) {
      const double ee = s.e[0] * s.e[0] + s.e[1] * s.e[1] + s.e[2] * s.e[2];
      const double q = 2.0 * mp.mu * sqrt(1.5 * ee);
      const double w3q = 3.0 * mp.mu / q;
      const double xe = Xd[0] * s.e[0] + Xd[1] * s.e[1] + Xd[2] * s.e[2];
      const double hterm = MB ? Hb * 2.0 * mp.mu * s.c * ee : (s.hactive ? Lb * s.gp * 2.0 * mp.mu * s.c * ee : 0.0);
      const double base = s.g * 2.0 * mp.mu * xe + hterm;
      gsum[1] = -w3q * s.ddg_s0 * base;
      gsum[2] = -w3q * s.ddg_visc * base;
    }
    if (MB) {
      sW.put(Pb);
      mb_adjoint_extra<VOCE>(a, pidc, gq, pt, sG, phi, sW, Hb, Fu, phib);
    }
    f0 = phib;
  }
  if (MB) bad |= pt && xbad;
  // point coefficients into Qi (bufB is free: every thread has read its values)
  if (pt) {
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      double b[3];
      phys_to_ref<GEO>(f < 3 ? Fu + 3 * f : f1, ih, gA, b);
#pragma unroll
      for (int K = 0; K < 3; ++K) bufB[qslot<true>(f, 1 + K) * Q3 + ql] = b[K];
    }
    bufB[qslot<true>(3, 0) * Q3 + ql] = f0;
  }
  __syncthreads();
  sf5_bwd<double, DevTables, P, Q, 4, true>(bufB, bufA, tabs);
  if (TAB)
    store_elem_tab<double, P>(bufA, e, a.evec);
  else if (EV)
    store_ext<double, P, 4>(bufA, a.m, g, a.evec);
  else
    scatter_elem<double, P, 4>(bufA, a.m, a.nx1, a.ny1, a.n_nodes, g, a.out);
  if (MODE == M_ADJ) {
    // deterministic per-phase sums of the element's point partials: a butterfly in each
    // wave, then the two wave sums in wave order
    const int nv = 3 * a.nph;
    const int l = t & 63, wv = t >> 6;
    for (int idx = 0; idx < nv; ++idx) {
      const int ph = idx / 3, k = idx - 3 * ph;
      const double gk = k == 0 ? gsum[0] : (k == 1 ? gsum[1] : gsum[2]);
      double v = (pt && pid == ph) ? gk : 0.0;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if (l == 0 && nv <= 24) red[wv * nv + idx] = v;
      if (nv > 24) {
        // many phases: serialise through one LDS slot pair
        if (l == 0) red[wv] = v;
        __syncthreads();
        if (t == 0) a.gpart[e * nv + idx] = red[0] + red[1];
        __syncthreads();
      }
    }
    if (nv <= 24) {
      __syncthreads();
      if (t < nv) a.gpart[e * nv + t] = red[t] + red[nv + t];
    }
  }
  if (bad) a.flag[0] = 1;
  if (bad_pid) a.flag[1] = 1;
}

// FP32 level apply (direction on a level with PC nodes per direction, kinematics on the
// fine order-4 lattice) on order-4 fine elements.
template <typename V> struct TablesOf;
template <> struct TablesOf<float> { using type = DevTablesF; };
template <> struct TablesOf<double> { using type = DevTables; };

// EV: all elements in one launch, the level's element vectors stored to the extended
// node grid a.ebuf [4][nz PC][ny PC][nx PC] (summed per node by k_gather_ext).
template <typename V, int PC, bool MB, bool GEO = false, bool EV = false>
__global__ __launch_bounds__(NT5, 2) void k_a32_q4(LinApplyArgs<V> a, int colour,
                                                   const typename TablesOf<V>::type* __restrict__ tabs) {
  using Tab = typename TablesOf<V>::type;
  constexpr int PF = 5, Q = 5, Q3 = 125;
  using L = Q5Lds<PF, Q, true>;  // compact point arrays for the direction (as k_op64_q4)
  __shared__ V bufA[L::A];
  __shared__ V bufB[L::B];
  ElemGeom g;
  if (!(EV ? xcd_elem_all(a.m, blockIdx.x, g) : xcd_elem(a.m, colour, blockIdx.x, g))) return;  // padding (uniform)
  const int t = threadIdx.x;
  const bool pt = t < Q3;
  const int ql = pt ? t : 0;
  const int qx = ql % Q, qy = (ql / Q) % Q, qz = ql / (Q * Q);
  const int64_t e = (int64_t)g.ex + (int64_t)a.m.nx * (g.ey + (int64_t)a.m.ny * g.ez);
  const int64_t gq = e * Q3 + ql;
  LinRecordT<V> rc;
#pragma unroll
  for (int k = 0; k < REC_N; ++k) rc.v[k] = pt ? a.rec.rec[k * a.n_q + gq] : V(0);
  rc.flags = pt ? a.rec.flags[gq] : 0;
  const int pid = pt ? a.phase[gq] : 0;
  const V ih[3] = {(V)a.m.ih[0], (V)a.m.ih[1], (V)a.m.ih[2]};
  V wdet = tabs->w[Q][qx] * tabs->w[Q][qy] * tabs->w[Q][qz] * (V)a.m.jdet;
  // mapped elements: the point's J^-1 and weight
  double gA[GEO ? 9 : 1];
  if (GEO) {
#pragma unroll
    for (int k = 0; k < 9; ++k) gA[k] = pt ? a.qd[k * a.n_q + gq] : 0.0;
    wdet = pt ? (V)a.qd[9 * a.n_q + gq] : V(0);
  }
  gather_nodes<V, V, PF, 3>(a.z32, a.fine.n_nodes, elem_node<PF>(a.fine.nx1, a.fine.ny1, g), bufA);
  __syncthreads();
  sf5_fwd<V, Tab, PF, Q, 3>(bufA, bufB, tabs);
  V G[9];
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    if (GEO)
      map_grad<V>((double)bufB[(4 * f + 1) * Q3 + ql], (double)bufB[(4 * f + 2) * Q3 + ql],
                  (double)bufB[(4 * f + 3) * Q3 + ql], gA, G + 3 * f);
    else
#pragma unroll
      for (int J = 0; J < 3; ++J) G[3 * f + J] = bufB[(4 * f + 1 + J) * Q3 + ql] * ih[J];
  }
  __syncthreads();
  gather_nodes<V, V, PC, 4>(a.dz, a.lev.n_nodes, elem_node<PC>(a.lev.nx1, a.lev.ny1, g), bufA);
  __syncthreads();
  sf5_fwd<V, Tab, PC, Q, 4, true>(bufA, bufB, tabs);
  V W[9], wphi, gw[3];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    V* out = f < 3 ? W + 3 * f : gw;
    if (GEO)
      map_grad<V>((double)bufB[qslot<true>(f, 1) * Q3 + ql], (double)bufB[qslot<true>(f, 2) * Q3 + ql],
                  (double)bufB[qslot<true>(f, 3) * Q3 + ql], gA, out);
    else
#pragma unroll
      for (int J = 0; J < 3; ++J) out[J] = bufB[qslot<true>(f, 1 + J) * Q3 + ql] * ih[J];
  }
  wphi = bufB[qslot<true>(3, 0) * Q3 + ql];
  __syncthreads();
  const int pidc = pid < a.nph ? pid : 0;
  const MatParams<V> mp = a.mats[pidc];
  QPState<V> s;
  qp_state_lin<V>(mp, G, rc, s);
  V Fu[9], dL;
  lin_tangent<V, MB>(a.rec, a.n_q, a.xmats, a.n_extra, mp, s, pidc, gq, pt, G, W, wphi, Fu, dL);
  const V kfg = a.fr.kf * mp.Gc;
  if (pt && GEO) {
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      double fl[3], b[3];
#pragma unroll
      for (int J = 0; J < 3; ++J) fl[J] = f < 3 ? (double)(wdet * Fu[3 * f + J]) : (double)(wdet * kfg * gw[J]);
      phys_to_ref<true>(fl, nullptr, gA, b);
#pragma unroll
      for (int K = 0; K < 3; ++K) bufB[qslot<true>(f, 1 + K) * Q3 + ql] = (V)b[K];
    }
    bufB[qslot<true>(3, 0) * Q3 + ql] = wdet * a.fr.s_phi * dL;
  } else if (pt) {
#pragma unroll
    for (int f = 0; f < 3; ++f)
#pragma unroll
      for (int J = 0; J < 3; ++J) bufB[qslot<true>(f, 1 + J) * Q3 + ql] = wdet * Fu[3 * f + J] * ih[J];
    bufB[qslot<true>(3, 0) * Q3 + ql] = wdet * a.fr.s_phi * dL;
#pragma unroll
    for (int J = 0; J < 3; ++J) bufB[qslot<true>(3, 1 + J) * Q3 + ql] = wdet * kfg * gw[J] * ih[J];
  }
  __syncthreads();
  sf5_bwd<V, Tab, PC, Q, 4, true>(bufB, bufA, tabs);
  if (EV)
    store_ext<V, PC, 4>(bufA, a.m, g, a.ebuf);
  else
    scatter_elem<V, PC, 4>(bufA, a.m, a.lev.nx1, a.lev.ny1, a.lev.n_nodes, g, a.out);
}


// Linearised level apply on an order-2 fine mesh (3 nodes, 3 Gauss points per direction)
// in row layout, without extra branches and on box elements: the k_a32_q4 scheme with a
// brick of 2 x 2 x 2 elements per 256-thread workgroup. Each element has 32 threads for
// the pointwise function (27 points) and its own LDS buffers, and the sum factorisation
// tasks of the eight elements (a (field, line) each) are spread over the workgroup, so
// that no contraction is padded from 3 to 4 points. The element vectors go to the brick
// sums in the padded 4^3 lane layout (store_brick4), then k_gather_ext<V, 2 PC - 1>.
template <typename V, int PC>
__global__ __launch_bounds__(NT, 2) void k_a32_q2r(LinApplyArgs<V> a, const typename TablesOf<V>::type* __restrict__ tabs) {
  using Tab = typename TablesOf<V>::type;
  constexpr int PF = 3, Q = 3, Q3 = 27, NE = 8, PC3 = PC * PC * PC;
  static_assert(PC <= PF && NE * 32 == NT, "eight elements of 32 threads");
  using L = Q5Lds<PF, Q, true>;
  static_assert(NE * 4 * 64 <= NE * L::B, "the element vectors reuse the point buffers");
  __shared__ V bufA[NE * L::A];
  __shared__ V bufB[NE * L::B];
  V* ev = bufB;  // element vectors, once the transposed passes have left the point buffers
  const int brick = xcd_brick_all(a.m, blockIdx.x);
  if (brick < 0) return;  // padding workgroup (uniform)
  const BrickGeom bg = decode_brick_lin(a.m, brick);
  const int t = threadIdx.x, slot = t >> 5, n = t & 31;
  const int sx = slot & 1, sy = (slot >> 1) & 1, sz = slot >> 2;
  const bool ein = sx < bg.nex && sy < bg.ney && sz < bg.nez;  // the slot holds an element
  const bool pt = ein && n < Q3;
  const int ql = pt ? n : 0;
  const int qx = ql % Q, qy = (ql / Q) % Q, qz = ql / (Q * Q);
  const ElemGeom g{bg.ex0 + sx, bg.ey0 + sy, bg.ez0 + sz};
  const int64_t e = (int64_t)g.ex + (int64_t)a.m.nx * (g.ey + (int64_t)a.m.ny * g.ez);
  const int64_t gq = e * Q3 + ql;
  V* A = bufA + slot * L::A;
  V* B = bufB + slot * L::B;
  LinRecordT<V> rc;
#pragma unroll
  for (int k = 0; k < REC_N; ++k) rc.v[k] = pt ? a.rec.rec[k * a.n_q + gq] : V(0);
  rc.flags = pt ? a.rec.flags[gq] : 0;
  const int pid = pt ? a.phase[gq] : 0;
  const V ih[3] = {(V)a.m.ih[0], (V)a.m.ih[1], (V)a.m.ih[2]};
  const V wdet = tabs->w[Q][qx] * tabs->w[Q][qy] * tabs->w[Q][qz] * (V)a.m.jdet;
  // the fine displacement mirror at the element's 27 nodes (thread n owns node n)
  if (ein && n < PF * PF * PF) {
    const int64_t gn = lattice_node<PF>(a.fine.nx1, a.fine.ny1, g, n);
    V v[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) v[f] = a.z32[f * a.fine.n_nodes + gn];
#pragma unroll
    for (int f = 0; f < 3; ++f) A[f * PF * PF * PF + n] = v[f];
  }
  __syncthreads();
  sf5_fwd<V, Tab, PF, Q, 3, false, true, NE, NT>(bufA, bufB, tabs, L::A, L::B);
  V G[9];
#pragma unroll
  for (int f = 0; f < 3; ++f)
#pragma unroll
    for (int J = 0; J < 3; ++J) G[3 * f + J] = B[(4 * f + 1 + J) * Q3 + ql] * ih[J];
  __syncthreads();
  // the level direction at the element's PC^3 nodes
  if (ein && n < PC3) {
    const int64_t gn = lattice_node<PC>(a.lev.nx1, a.lev.ny1, g, n);
    V v[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) v[f] = a.dz[f * a.lev.n_nodes + gn];
#pragma unroll
    for (int f = 0; f < 4; ++f) A[f * PC3 + n] = v[f];
  }
  __syncthreads();
  sf5_fwd<V, Tab, PC, Q, 4, true, true, NE, NT>(bufA, bufB, tabs, L::A, L::B);
  V W[9], wphi, gw[3];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    V* out = f < 3 ? W + 3 * f : gw;
#pragma unroll
    for (int J = 0; J < 3; ++J) out[J] = B[qslot<true>(f, 1 + J) * Q3 + ql] * ih[J];
  }
  wphi = B[qslot<true>(3, 0) * Q3 + ql];
  __syncthreads();
  const int pidc = pid < a.nph ? pid : 0;
  const MatParams<V> mp = a.mats[pidc];
  QPState<V> s;
  qp_state_lin<V>(mp, G, rc, s);
  V Fu[9], dL;
  lin_tangent<V, false>(a.rec, a.n_q, a.xmats, a.n_extra, mp, s, pidc, gq, pt, G, W, wphi, Fu, dL);
  const V kfg = a.fr.kf * mp.Gc;
  if (pt) {
#pragma unroll
    for (int f = 0; f < 3; ++f)
#pragma unroll
      for (int J = 0; J < 3; ++J) B[qslot<true>(f, 1 + J) * Q3 + ql] = wdet * Fu[3 * f + J] * ih[J];
    B[qslot<true>(3, 0) * Q3 + ql] = wdet * a.fr.s_phi * dL;
#pragma unroll
    for (int J = 0; J < 3; ++J) B[qslot<true>(3, 1 + J) * Q3 + ql] = wdet * kfg * gw[J] * ih[J];
  }
  __syncthreads();
  sf5_bwd<V, Tab, PC, Q, 4, true, NE, NT>(bufB, bufA, tabs, L::B, L::A);
  // element vectors into the padded lane layout of the brick sums (node a = i + 4 j + 16 k)
  if (ein && n < PC3) {
    const int i = n % PC, j = (n / PC) % PC, k = n / (PC * PC);
#pragma unroll
    for (int f = 0; f < 4; ++f) ev[(slot * 4 + f) * 64 + i + 4 * j + 16 * k] = A[f * PC3 + n];
  }
  __syncthreads();
  store_brick4<V, PC, 4>(ev, a.m, bg, a.ebuf);
}


// FP64 residual / Jacobian / adjoint on order-2 box elements without extra branches, in
// row layout: a brick of 2 x 2 x 2 elements per 256-thread workgroup, 32 threads per
// element for the pointwise function (27 points), the eight elements' sum factorisation
// tasks spread over the workgroup through LDS (no contraction padded from 3 to 4 points).
// Brick sums to the brick buffer (store_brick4), then k_gather_ext<double, 5>; the
// adjoint's per-phase parameter partials are summed per brick in a fixed order.
template <int MODE, bool VOCE>
__global__ __launch_bounds__(NT, 2) void k_op64_q2r(OpArgs a, DevTables* __restrict__ tabs) {
  constexpr int P = 3, Q = 3, Q3 = 27, NE = 8;
  static_assert(NE * 32 == NT, "eight elements of 32 threads");
  using L = Q5Lds<P, Q, true>;
  static_assert(NE * 4 * 64 <= NE * L::B, "the element vectors reuse the point buffers");
  __shared__ double bufA[NE * L::A];
  __shared__ double bufB[NE * L::B];
  __shared__ double red[MODE == M_ADJ ? NT : 1];
  double* ev = bufB;  // element vectors, once the transposed passes have left the point buffers
  const int brick = xcd_brick_all(a.m, blockIdx.x);
  if (brick < 0) return;  // padding workgroup (uniform)
  const BrickGeom bg = decode_brick_lin(a.m, brick);
  const int t = threadIdx.x, slot = t >> 5, n = t & 31, l = t & 63, wv = t >> 6;
  const int sx = slot & 1, sy = (slot >> 1) & 1, sz = slot >> 2;
  const bool ein = sx < bg.nex && sy < bg.ney && sz < bg.nez;  // the slot holds an element
  const bool pt = ein && n < Q3;
  const int ql = pt ? n : 0;
  const int qx = ql % Q, qy = (ql / Q) % Q, qz = ql / (Q * Q);
  const ElemGeom g{bg.ex0 + sx, bg.ey0 + sy, bg.ez0 + sz};
  const int64_t e = (int64_t)g.ex + (int64_t)a.m.nx * (g.ey + (int64_t)a.m.ny * g.ez);
  const int64_t gq = e * Q3 + ql;
  const int64_t gn = (ein && n < Q3) ? lattice_node<P>(a.nx1, a.ny1, g, n) : -1;  // thread n owns node n
  double* A = bufA + slot * L::A;
  double* B = bufB + slot * L::B;
  // per-point state, issued before the gathers
  double st[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) st[k] = pt ? a.state[k * a.n_q + gq] : 0.0;
  const int pid = pt ? a.phase[gq] : 0;
  const double ih[3] = {a.m.ih[0], a.m.ih[1], a.m.ih[2]};
  const double wdet = tabs->w[Q][qx] * tabs->w[Q][qy] * tabs->w[Q][qz] * a.m.jdet;
  if (gn >= 0) {
    double v[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) v[f] = a.z[f * a.n_nodes + gn];
#pragma unroll
    for (int f = 0; f < 4; ++f) A[f * Q3 + n] = v[f];
  }
  __syncthreads();
  sf5_fwd<double, DevTables, P, Q, 4, true, true, NE, NT>(bufA, bufB, tabs, L::A, L::B);
  double G[9], phi, gphi[3];
#pragma unroll
  for (int f = 0; f < 4; ++f)
#pragma unroll
    for (int J = 0; J < 3; ++J) (f < 3 ? G + 3 * f : gphi)[J] = B[qslot<true>(f, 1 + J) * Q3 + ql] * ih[J];
  phi = B[qslot<true>(3, 0) * Q3 + ql];
  double phin = 0.0;
  __syncthreads();
  if (MODE == M_RES) {
    if (gn >= 0) A[n] = a.phin[gn];
    __syncthreads();
    sf5_fwd<double, DevTables, P, Q, 1, false, false, NE, NT>(bufA, bufB, tabs, L::A, L::B);
    phin = B[ql];
    __syncthreads();
  }
  const bool bad_pid = pt && pid >= a.nph;  // an id outside the phase table raises the phase flag
  const int pidc = pid < a.nph ? pid : 0;
  const MatParams<double> mp = a.mats[pidc];
  QPState<double> s;
  qp_state<double, VOCE>(mp, a.fr, G, phi, phin, st, s);
  const bool bad = pt && s.bad;
  double W[9], wphi = 0.0, gw[3] = {0.0, 0.0, 0.0};
  if (MODE != M_RES) {
    if (gn >= 0) {
      double v[4];
#pragma unroll
      for (int f = 0; f < 4; ++f) v[f] = a.w[f * a.n_nodes + gn];
#pragma unroll
      for (int f = 0; f < 4; ++f) A[f * Q3 + n] = v[f];
    }
    __syncthreads();
    sf5_fwd<double, DevTables, P, Q, 4, true, true, NE, NT>(bufA, bufB, tabs, L::A, L::B);
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
      for (int J = 0; J < 3; ++J) (f < 3 ? W + 3 * f : gw)[J] = B[qslot<true>(f, 1 + J) * Q3 + ql] * ih[J];
    wphi = B[qslot<true>(3, 0) * Q3 + ql];
    __syncthreads();
  }
  const double kfg = a.fr.kf * mp.Gc;
  double Fu[9], f0, f1[3];
  double gsum[3] = {0.0, 0.0, 0.0};
  if (MODE == M_RES) {
    piola<double>(s, Fu);
#pragma unroll
    for (int k = 0; k < 9; ++k) Fu[k] *= wdet;
    f0 = wdet * a.fr.s_phi * s.L;
#pragma unroll
    for (int J = 0; J < 3; ++J) f1[J] = wdet * kfg * gphi[J];
  } else if (MODE == M_JAC) {
    double dL;
    qp_tangent<double>(mp, s, W, wphi, Fu, dL);
#pragma unroll
    for (int k = 0; k < 9; ++k) Fu[k] *= wdet;
    f0 = wdet * a.fr.s_phi * dL;
#pragma unroll
    for (int J = 0; J < 3; ++J) f1[J] = wdet * kfg * gw[J];
  } else {
    double Pb[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) Pb[k] = wdet * W[k];
    const double f0b = wdet * wphi;
    const double Lb = a.fr.s_phi * f0b;
    double phib, Xd[3];
    qp_tangent_T<double>(mp, s, Pb, Lb, Fu, phib, Xd);
#pragma unroll
    for (int J = 0; J < 3; ++J) f1[J] = kfg * wdet * gw[J];
    const double alpha_p = (a.fr.at == 2) ? 2.0 * phi : 1.0;
    gsum[0] = alpha_p * a.fr.inv_c0l0 * Lb + a.fr.kf * wdet * (gphi[0] * gw[0] + gphi[1] * gw[1] + gphi[2] * gw[2]);
    if (s.plastic) {
      const double ee = s.e[0] * s.e[0] + s.e[1] * s.e[1] + s.e[2] * s.e[2];
      const double qv = 2.0 * mp.mu * sqrt(1.5 * ee);
      const double w3q = 3.0 * mp.mu / qv;
      const double xe = Xd[0] * s.e[0] + Xd[1] * s.e[1] + Xd[2] * s.e[2];
      const double hterm = s.hactive ? Lb * s.gp * 2.0 * mp.mu * s.c * ee : 0.0;
      const double base = s.g * 2.0 * mp.mu * xe + hterm;
      gsum[1] = -w3q * s.ddg_s0 * base;
      gsum[2] = -w3q * s.ddg_visc * base;
    }
    f0 = phib;
    if (!pt) gsum[0] = gsum[1] = gsum[2] = 0.0;
  }
  // point coefficients into the point arrays (every thread has read its values)
  if (pt) {
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
      for (int K = 0; K < 3; ++K) B[qslot<true>(f, 1 + K) * Q3 + ql] = (f < 3 ? Fu[3 * f + K] : f1[K]) * ih[K];
    B[qslot<true>(3, 0) * Q3 + ql] = f0;
  }
  __syncthreads();
  sf5_bwd<double, DevTables, P, Q, 4, true, NE, NT>(bufB, bufA, tabs, L::B, L::A);
  // element vectors into the padded lane layout of the brick sums (node a = i + 4 j + 16 k)
  if (gn >= 0) {
    const int i = n % P, j = (n / P) % P, k = n / (P * P);
#pragma unroll
    for (int f = 0; f < 4; ++f) ev[(slot * 4 + f) * 64 + i + 4 * j + 16 * k] = A[f * Q3 + n];
  }
  if (MODE == M_ADJ) {
    // deterministic per-phase reduction: butterfly inside each wave, wave sums in order
    const int nv = 3 * a.nph;
    if (nv * (NT / 64) <= NT) {
      for (int idx = 0; idx < nv; ++idx) {
        const int ph = idx / 3, k = idx - 3 * ph;
        double v = (pt && pid == ph) ? (k == 0 ? gsum[0] : (k == 1 ? gsum[1] : gsum[2])) : 0.0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (l == 0) red[wv * nv + idx] = v;
      }
      __syncthreads();
      if (t < nv) {
        double r = red[t];
        for (int w = 1; w < NT / 64; ++w) r += red[w * nv + t];
        a.gpart[(int64_t)(a.brick_base + brick) * nv + t] = r;
      }
    } else {
      for (int ph = 0; ph < a.nph; ++ph) {
        for (int k = 0; k < 3; ++k) {
          red[t] = (pt && pid == ph) ? (k == 0 ? gsum[0] : (k == 1 ? gsum[1] : gsum[2])) : 0.0;
          __syncthreads();
          for (int stp = NT / 2; stp > 0; stp >>= 1) {
            if (t < stp) red[t] += red[t + stp];
            __syncthreads();
          }
          if (t == 0) a.gpart[((int64_t)(a.brick_base + brick) * a.nph + ph) * 3 + k] = red[0];
          __syncthreads();
        }
      }
    }
  }
  __syncthreads();
  store_brick4<double, P, 4>(ev, a.m, bg, a.ebuf);
  if (bad) a.flag[0] = 1;
  if (bad_pid) a.flag[1] = 1;
}

}  // namespace pfmf
