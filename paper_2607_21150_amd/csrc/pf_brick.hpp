// Element-brick machinery shared by the operator kernels (device side).
//
// A workgroup owns a brick of up to 2x2x2 elements of a structured mesh. The
// brick's nodal values are staged in LDS once (gather E P z), the elements are
// processed in rounds (one thread per quadrature point), their element vectors
// are kept in LDS, and each brick node sums the contributions of the brick's
// elements in a fixed order. Bricks are launched in 8 colours by the parity of
// their brick coordinates; bricks of one colour share no node, so the write of
// a brick's nodes to the global vector is race-free. A node on a brick face is
// stored by the first colour that touches it and accumulated by the later ones,
// which makes the scatter-add (E^T P^T) deterministic without atomics.
//
// Sum factorisation (Section 4, B_I and B_xi) runs through LDS with one pass per
// direction: x and y passes write LDS arrays, the z pass is evaluated by the
// thread that owns the quadrature point. The transposed passes run in the
// opposite order and land in the element vector.
#pragma once
#include <hip/hip_runtime.h>

namespace pfmf {

constexpr int NT = 256;  // threads per workgroup

// 1-D tables per (P nodes, Q points): B[q][i], D[q][i], w[q] (index [P][Q]); G[Q][q][m]
// = derivative at Gauss point q of the Lagrange polynomial through the Q Gauss points that
// is 1 at point m (collocated differentiation of values already at the points).
struct DevTables {
  double B[6][6][5][5];
  double D[6][6][5][5];
  double w[6][5];
  double G[6][5][5];
};
struct DevTablesF {
  float B[6][6][5][5];
  float D[6][6][5][5];
  float w[6][5];
  float G[6][5][5];
};

struct BrickGeom {
  int bx, by, bz;        // brick coordinates
  int nex, ney, nez;     // elements in this brick per direction (1 or 2)
  int ex0, ey0, ez0;     // first element
  bool last_x, last_y, last_z;
};

struct MeshDev {
  int nx, ny, nz;
  int nbx, nby, nbz;     // bricks per direction
  double hx, hy, hz;
  double ih[3];          // 2 / h per direction (reference-to-physical gradient factor)
  double jdet;           // hx hy hz / 8 (affine Jacobian determinant)
};

__device__ inline BrickGeom decode_brick(const MeshDev& m, int colour, int b) {
  const int cx = colour & 1, cy = (colour >> 1) & 1, cz = (colour >> 2) & 1;
  const int CX = (m.nbx - cx + 1) / 2, CY = (m.nby - cy + 1) / 2;
  BrickGeom g;
  g.bx = cx + 2 * (b % CX);
  g.by = cy + 2 * ((b / CX) % CY);
  g.bz = cz + 2 * (b / (CX * CY));
  g.ex0 = 2 * g.bx;
  g.ey0 = 2 * g.by;
  g.ez0 = 2 * g.bz;
  g.nex = min(2, m.nx - g.ex0);
  g.ney = min(2, m.ny - g.ey0);
  g.nez = min(2, m.nz - g.ez0);
  g.last_x = g.bx == m.nbx - 1;
  g.last_y = g.by == m.nby - 1;
  g.last_z = g.bz == m.nbz - 1;
  return g;
}

// XCD-aware workgroup order. Workgroups are dispatched to the 8 XCDs round-robin by id,
// and each XCD has its own L2. Within one colour only bricks of the same x-row share
// cache lines of the nodal vectors (a 128-byte line spans 16 nodes, a brick 7), so the
// bricks of one x-row are given ids 8 apart: they run on one XCD, back to back, and
// re-read the shared lines from its L2. xcd_grid is the padded grid size;
// xcd_brick maps an id to the brick index of decode_brick, or -1 for padding.
__host__ __device__ inline int xcd_grid(int nbx, int nby, int nbz, int colour) {
  const int cx = colour & 1, cy = (colour >> 1) & 1, cz = (colour >> 2) & 1;
  const int CX = (nbx - cx + 1) / 2, CY = (nby - cy + 1) / 2, CZ = (nbz - cz + 1) / 2;
  const int rows = CY * CZ;
  return CX == 0 || rows == 0 ? 0 : ((rows + 7) / 8) * 8 * CX;
}
__device__ inline int xcd_brick(const MeshDev& m, int colour, int id) {
  const int cx = colour & 1, cy = (colour >> 1) & 1, cz = (colour >> 2) & 1;
  const int CX = (m.nbx - cx + 1) / 2, CY = (m.nby - cy + 1) / 2, CZ = (m.nbz - cz + 1) / 2;
  const int t = id >> 3;
  const int row = (t / CX) * 8 + (id & 7);
  return row < CY * CZ ? (t % CX) + CX * row : -1;
}

// All bricks in one launch (the brick-buffer scatter): the same XCD-aware order over
// the whole brick grid. Returns the linear brick index bx + nbx (by + nby bz), or -1.
__host__ __device__ inline int xcd_grid_all(int nbx, int nby, int nbz) {
  const int rows = nby * nbz;
  return ((rows + 7) / 8) * 8 * nbx;
}
__device__ inline int xcd_brick_all(const MeshDev& m, int id) {
  const int t = id >> 3;
  const int row = (t / m.nbx) * 8 + (id & 7);
  return row < m.nby * m.nbz ? (t % m.nbx) + m.nbx * row : -1;
}
__device__ inline BrickGeom decode_brick_lin(const MeshDev& m, int b) {
  BrickGeom g;
  g.bx = b % m.nbx;
  g.by = (b / m.nbx) % m.nby;
  g.bz = b / (m.nbx * m.nby);
  g.ex0 = 2 * g.bx;
  g.ey0 = 2 * g.by;
  g.ez0 = 2 * g.bz;
  g.nex = min(2, m.nx - g.ex0);
  g.ney = min(2, m.ny - g.ey0);
  g.nez = min(2, m.nz - g.ez0);
  g.last_x = g.bx == m.nbx - 1;
  g.last_y = g.by == m.nby - 1;
  g.last_z = g.bz == m.nbz - 1;
  return g;
}

// Table restriction: groups of 8 consecutive elements, XCD-aware. Workgroup id w runs on
// XCD w % 8; group (w % 8) * per + w / 8 gives every XCD one contiguous range of groups,
// processed in order, so elements that are neighbours in the element order share its L2.
__host__ __device__ inline int xcd_grid_groups(int n_groups) { return ((n_groups + 7) / 8) * 8; }
__device__ inline int xcd_group(int n_groups, int id) {
  const int per = (n_groups + 7) / 8;
  const int gr = (id & 7) * per + (id >> 3);
  return gr < n_groups ? gr : -1;
}

__host__ __device__ inline int bricks_in_colour(int nbx, int nby, int nbz, int colour) {
  const int cx = colour & 1, cy = (colour >> 1) & 1, cz = (colour >> 2) & 1;
  return ((nbx - cx + 1) / 2) * ((nby - cy + 1) / 2) * ((nbz - cz + 1) / 2);
}

// Stage NF nodal fields of the brick (order p = P-1) into LDS arrays dst[f][NB^3].
template <typename T, typename S, int P, int NF>
__device__ inline void stage_brick(const S* __restrict__ src, int64_t n_nodes, int nx1, int ny1,
                                   const BrickGeom& g, T* dst) {
  constexpr int p = P - 1, NB = 2 * P - 1, NB3 = NB * NB * NB;
  const int mx = g.nex * p + 1, my = g.ney * p + 1, mz = g.nez * p + 1;
  for (int t = threadIdx.x; t < NB3; t += NT) {
    const int lx = t % NB, ly = (t / NB) % NB, lz = t / (NB * NB);
    if (lx < mx && ly < my && lz < mz) {
      const int64_t gi = (int64_t)(g.ex0 * p + lx) + (int64_t)nx1 * ((g.ey0 * p + ly) + (int64_t)ny1 * (g.ez0 * p + lz));
#pragma unroll
      for (int f = 0; f < NF; ++f) dst[f * NB3 + t] = (T)src[f * n_nodes + gi];
    }
  }
}

// Sum the element vectors ev[slot][f][P^3] into brick nodes and write them to
// dst[f][n_nodes]: store where this colour is the first to touch the node,
// accumulate otherwise.
template <typename T, int P, int NF>
__device__ inline void scatter_brick(const T* ev, const MeshDev& m, int nx1, int ny1, int64_t n_nodes,
                                     const BrickGeom& g, T* __restrict__ dst) {
  constexpr int p = P - 1, NB = 2 * P - 1, NB3 = NB * NB * NB, P3 = P * P * P;
  const int mx = g.nex * p + 1, my = g.ney * p + 1, mz = g.nez * p + 1;
  const int px = g.bx & 1, py = g.by & 1, pz = g.bz & 1;
  for (int t = threadIdx.x; t < NB3; t += NT) {
    const int lx = t % NB, ly = (t / NB) % NB, lz = t / (NB * NB);
    if (!(lx < mx && ly < my && lz < mz)) continue;
    T acc[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[f] = T(0);
    // fixed order over the brick's element slots (sz, sy, sx)
#pragma unroll
    for (int sz = 0; sz < 2; ++sz) {
      const int k = lz - sz * p;
      if (k < 0 || k > p || sz >= g.nez) continue;
#pragma unroll
      for (int sy = 0; sy < 2; ++sy) {
        const int j = ly - sy * p;
        if (j < 0 || j > p || sy >= g.ney) continue;
#pragma unroll
        for (int sx = 0; sx < 2; ++sx) {
          const int i = lx - sx * p;
          if (i < 0 || i > p || sx >= g.nex) continue;
          const int slot = sx + 2 * sy + 4 * sz;
          const int a = i + P * (j + P * k);
#pragma unroll
          for (int f = 0; f < NF; ++f) acc[f] += ev[(slot * NF + f) * P3 + a];
        }
      }
    }
    const bool shx = (lx == 0 && g.bx > 0) || (lx == mx - 1 && !g.last_x);
    const bool shy = (ly == 0 && g.by > 0) || (ly == my - 1 && !g.last_y);
    const bool shz = (lz == 0 && g.bz > 0) || (lz == mz - 1 && !g.last_z);
    const bool store = !((shx && px) || (shy && py) || (shz && pz));
    const int64_t gi = (int64_t)(g.ex0 * p + lx) + (int64_t)nx1 * ((g.ey0 * p + ly) + (int64_t)ny1 * (g.ez0 * p + lz));
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      T* d = dst + f * n_nodes + gi;
      if (store) *d = acc[f];
      else *d += acc[f];
    }
  }
}

// ---------------------------------------------------------------------------
// Sum factorisation through LDS for one round of ER element slots.
// Layouts (x fastest): nodal [el][k][j][i] (brick LDS), after x-pass
// [el][k][j][qx], after y-pass [el][k][qy][qx], quadrature [el][qz][qy][qx].
// ---------------------------------------------------------------------------

template <typename T> struct TabRef {
  const T* B;  // [Q][P] (LDS copy)
  const T* D;
};

// x and y passes of the forward interpolation for one field.
//   grad: also produce the derivative intermediates.
// Outputs: ybb = B_y B_x U, ydb = D_y B_x U, ybd = B_y D_x U  (each [ER][P][Q][Q])
template <typename T, int P, int Q, int ER>
__device__ inline void fwd_xy(const T* Ub, int slot0, const BrickGeom& g, const TabRef<T>& tb, bool grad,
                              T* xb, T* xd, T* ybb, T* ydb, T* ybd) {
  constexpr int p = P - 1, NB = 2 * P - 1;
  constexpr int NX = ER * P * P * Q;
  for (int o = threadIdx.x; o < NX; o += NT) {
    const int qx = o % Q, j = (o / Q) % P, k = (o / (Q * P)) % P, el = o / (Q * P * P);
    const int slot = slot0 + el;
    const int sx = slot & 1, sy = (slot >> 1) & 1, sz = slot >> 2;
    const T* u = Ub + (sx * p) + NB * ((sy * p + j) + NB * (sz * p + k));
    T a = T(0), d = T(0);
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const T v = u[i];
      a += tb.B[qx * P + i] * v;
      d += tb.D[qx * P + i] * v;
    }
    xb[o] = a;
    if (grad) xd[o] = d;
  }
  __syncthreads();
  constexpr int NY = ER * P * Q * Q;
  for (int o = threadIdx.x; o < NY; o += NT) {
    const int qx = o % Q, qy = (o / Q) % Q, rest = o / (Q * Q);  // rest = k + P*el
    const T* s0 = xb + rest * (P * Q) + qx;
    const T* s1 = xd + rest * (P * Q) + qx;
    T bb = T(0), db = T(0), bd = T(0);
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const T v = s0[j * Q];
      bb += tb.B[qy * P + j] * v;
      if (grad) {
        db += tb.D[qy * P + j] * v;
        bd += tb.B[qy * P + j] * s1[j * Q];
      }
    }
    ybb[o] = bb;
    if (grad) {
      ydb[o] = db;
      ybd[o] = bd;
    }
  }
  __syncthreads();
}

// z pass at one quadrature point (el, qx, qy, qz) owned by the calling thread.
// Returns value and reference-coordinate gradient (xi_x, xi_y, xi_z).
template <typename T, int P, int Q>
__device__ inline void fwd_z(const T* ybb, const T* ydb, const T* ybd, int el, int qx, int qy, int qz,
                             const TabRef<T>& tb, bool grad, T& val, T* dxi) {
  const int base = el * (P * Q * Q) + qx + Q * qy;
  T v = T(0), dz = T(0), dy = T(0), dx = T(0);
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const T bz = tb.B[qz * P + k];
    const T w0 = ybb[base + k * Q * Q];
    v += bz * w0;
    if (grad) {
      dz += tb.D[qz * P + k] * w0;
      dy += bz * ydb[base + k * Q * Q];
      dx += bz * ybd[base + k * Q * Q];
    }
  }
  val = v;
  dxi[0] = dx;
  dxi[1] = dy;
  dxi[2] = dz;
}

// Transposed passes for one field: quadrature arrays f0 (value test), fx, fy, fz
// (reference-gradient tests), each [ER][Q^3], -> element vector rows
// ev[(slot*NF + f) * P^3 + a]. has_f0: whether f0 is present.
template <typename T, int P, int Q, int ER>
__device__ inline void bwd_field(const T* f0, const T* fx, const T* fy, const T* fz, bool has_f0, int slot0,
                                 int nslots, const TabRef<T>& tb, T* z0, T* zx, T* zy, T* y0, T* yx, T* ev,
                                 int NF, int f) {
  constexpr int P3 = P * P * P;
  // z^T: [el][k][qy][qx]
  constexpr int NZ = ER * P * Q * Q;
  for (int o = threadIdx.x; o < NZ; o += NT) {
    const int qx = o % Q, qy = (o / Q) % Q, k = (o / (Q * Q)) % P, el = o / (Q * Q * P);
    const int base = el * Q * Q * Q + qx + Q * qy;
    T a0 = T(0), ax = T(0), ay = T(0);
#pragma unroll
    for (int qz = 0; qz < Q; ++qz) {
      const int qi = base + qz * Q * Q;
      const T bz = tb.B[qz * P + k];
      a0 += tb.D[qz * P + k] * fz[qi];
      if (has_f0) a0 += bz * f0[qi];
      ax += bz * fx[qi];
      ay += bz * fy[qi];
    }
    z0[o] = a0;
    zx[o] = ax;
    zy[o] = ay;
  }
  __syncthreads();
  // y^T: [el][k][j][qx]
  constexpr int NY = ER * P * P * Q;
  for (int o = threadIdx.x; o < NY; o += NT) {
    const int qx = o % Q, j = (o / Q) % P, rest = o / (Q * P);  // rest = k + P*el
    const int base = rest * (Q * Q) + qx;
    T a0 = T(0), ax = T(0);
#pragma unroll
    for (int qy = 0; qy < Q; ++qy) {
      const T by = tb.B[qy * P + j];
      a0 += by * z0[base + qy * Q] + tb.D[qy * P + j] * zy[base + qy * Q];
      ax += by * zx[base + qy * Q];
    }
    y0[o] = a0;
    yx[o] = ax;
  }
  __syncthreads();
  // x^T -> element vector
  constexpr int NXo = ER * P * P * P;
  for (int o = threadIdx.x; o < NXo; o += NT) {
    const int i = o % P, rest = o / P;  // rest = j + P*(k + P*el)
    const int el = rest / (P * P);
    if (el >= nslots) continue;
    const int base = rest * Q;
    T a = T(0);
#pragma unroll
    for (int qx = 0; qx < Q; ++qx) a += tb.B[qx * P + i] * y0[base + qx] + tb.D[qx * P + i] * yx[base + qx];
    ev[((slot0 + el) * NF + f) * P3 + (o % P3)] = a;
  }
  __syncthreads();
}

}  // namespace pfmf
