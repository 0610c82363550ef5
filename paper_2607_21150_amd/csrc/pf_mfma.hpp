// Sum factorisation on the matrix cores for elements with at most 4 nodes and
// exactly 4 Gauss points per direction (Q3 fine level and the FP32 levels of a
// Q3 multigrid).
//
// One wavefront owns one element: lane l = a + 4 b + 16 c. v_mfma_f64_4x4x4f64
// (4 blocks) reads its A operand A[blk][i][k] at lane i + 4 blk + 16 k, its B
// operand B[blk][k][j] at lane j + 4 blk + 16 k and writes D[blk][i][j] at lane
// j + 4 blk + 16 i. With the element's data in A, one instruction contracts lane
// bits 4-5 and moves bits 0-1 there; with the data in B it contracts bits 4-5 in
// place. Bits 2-3 (the block) are brought to bits 4-5 by one lane permutation.
//
// Nodal layout: (x, y, z) = (bits 0-1, 2-3, 4-5).
// Point layout after the forward pass: (qx, qz, qy) = (bits 0-1, 2-3, 4-5).
// Forward: contract z (data in A), contract x (data in A), permute, contract y
// (data in B). Backward: contract qy (B), permute, contract qz (A), contract qx (A).
#pragma once
#include <hip/hip_runtime.h>

#include "pf_brick.hpp"
#include "pf_mg.hpp"
#include "pf_ops.hpp"
#include "pf_branch.hpp"
#include "pf_geom.hpp"
#include "pf_qf.hpp"

namespace pfmf {

__device__ inline double mfma4(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

// swap lane bits 2-3 with 4-5
__device__ inline double swap_blocks(double v) {
  const int l = threadIdx.x & 63;
  const int src = (l & 3) | ((l >> 4) << 2) | (((l >> 2) & 3) << 4);
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int rlo = __builtin_amdgcn_ds_bpermute(src << 2, lo);
  const int rhi = __builtin_amdgcn_ds_bpermute(src << 2, hi);
  return __hiloint2double(rhi, rlo);
}

// Per-lane basis operands of one (P, Q = 4) pair, zero-padded beyond P nodes.
//   fB = B[l%4][l/16] (B[q][node]), fD likewise; bB = B[l/16][l%4], bD likewise.
struct Basis4 {
  double fB, fD, bB, bD;
};

template <int P>
__device__ inline Basis4 load_basis4(const DevTables* __restrict__ t) {
  const int l = threadIdx.x & 63;
  const int a = l & 3, c = l >> 4;
  Basis4 b;
  b.fB = (c < P) ? t->B[P][4][a][c] : 0.0;
  b.fD = (c < P) ? t->D[P][4][a][c] : 0.0;
  b.bB = (a < P) ? t->B[P][4][c][a] : 0.0;
  b.bD = (a < P) ? t->D[P][4][c][a] : 0.0;
  return b;
}

// Basis operands of a (P, Q) pair with P, Q <= 4, zero-padded to 4 x 4: the padded
// points carry zero values and zero test functions.
template <int P, int Q>
__device__ inline Basis4 load_basis_pq(const DevTables* __restrict__ t) {
  const int l = threadIdx.x & 63;
  const int a = l & 3, c = l >> 4;
  Basis4 b;
  b.fB = (c < P && a < Q) ? t->B[P][Q][a][c] : 0.0;
  b.fD = (c < P && a < Q) ? t->D[P][Q][a][c] : 0.0;
  b.bB = (a < P && c < Q) ? t->B[P][Q][c][a] : 0.0;
  b.bD = (a < P && c < Q) ? t->D[P][Q][c][a] : 0.0;
  return b;
}

// Value of lane src (0..63) of the wave, for a double.
__device__ inline double lane_read(double v, int src) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  return __hiloint2double(__builtin_amdgcn_ds_bpermute(src << 2, hi), __builtin_amdgcn_ds_bpermute(src << 2, lo));
}

// Forward for NF fields in lockstep (independent chains interleaved): nodal
// values u[f] (layout x,y,z) -> value v[f] and reference gradient d[f][0..2] at
// the lane's point (layout qx,qz,qy). grad_mask / val_mask select the outputs.
template <int NF>
__device__ inline void sf4_fwd_n(const double* u, const Basis4& b, unsigned val_mask, unsigned grad_mask,
                                 double* v, double (*d)[3]) {
  double T[NF], Tz[NF], V2[NF], DX[NF], DZ[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    T[f] = mfma4(u[f], b.fB, 0.0);
    if ((grad_mask >> f) & 1) Tz[f] = mfma4(u[f], b.fD, 0.0);
  }
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    V2[f] = mfma4(T[f], b.fB, 0.0);
    if ((grad_mask >> f) & 1) {
      DX[f] = mfma4(T[f], b.fD, 0.0);
      DZ[f] = mfma4(Tz[f], b.fB, 0.0);
    }
  }
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    V2[f] = swap_blocks(V2[f]);
    if ((grad_mask >> f) & 1) {
      DX[f] = swap_blocks(DX[f]);
      DZ[f] = swap_blocks(DZ[f]);
    }
  }
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    if ((val_mask >> f) & 1) v[f] = mfma4(b.fB, V2[f], 0.0);
    if ((grad_mask >> f) & 1) {
      d[f][0] = mfma4(b.fB, DX[f], 0.0);
      d[f][1] = mfma4(b.fD, V2[f], 0.0);
      d[f][2] = mfma4(b.fB, DZ[f], 0.0);
    }
  }
}

// Backward for NF fields in lockstep: point coefficients f0[f] (value test, used
// where f0_mask is set) and f1[f][0..2] (reference-gradient tests) -> nodal
// contribution out[f] (layout x,y,z).
template <int NF>
__device__ inline void sf4_bwd_n(const double* f0, const double (*f1)[3], unsigned f0_mask, const Basis4& b,
                                 double* out) {
  double Z0[NF], Zx[NF], Zz[NF], Y0[NF], Yx[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    Z0[f] = mfma4(b.bD, f1[f][1], 0.0);
    Zx[f] = mfma4(b.bB, f1[f][0], 0.0);
    Zz[f] = mfma4(b.bB, f1[f][2], 0.0);
  }
#pragma unroll
  for (int f = 0; f < NF; ++f)
    if ((f0_mask >> f) & 1) Z0[f] = mfma4(b.bB, f0[f], Z0[f]);
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    Z0[f] = swap_blocks(Z0[f]);
    Zx[f] = swap_blocks(Zx[f]);
    Zz[f] = swap_blocks(Zz[f]);
  }
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    Y0[f] = mfma4(Zz[f], b.bD, 0.0);
    Yx[f] = mfma4(Zx[f], b.bB, 0.0);
  }
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    Y0[f] = mfma4(Z0[f], b.bB, Y0[f]);
    out[f] = mfma4(Yx[f], b.bD, 0.0);
  }
#pragma unroll
  for (int f = 0; f < NF; ++f) out[f] = mfma4(Y0[f], b.bB, out[f]);
}

// Sum the element vectors ev[slot][f][64] (lane-indexed nodes a = i + 4 j + 16 k)
// into the brick nodes and write them with the colour rule.
template <typename T, int P, int NF>
__device__ inline void scatter_brick4(const T* ev, const MeshDev& m, int nx1, int ny1, int64_t n_nodes,
                                      const BrickGeom& g, T* __restrict__ dst) {
  constexpr int p = P - 1, NB = 2 * P - 1, NB3 = NB * NB * NB;
  const int mx = g.nex * p + 1, my = g.ney * p + 1, mz = g.nez * p + 1;
  const int px = g.bx & 1, py = g.by & 1, pz = g.bz & 1;
  for (int t = threadIdx.x; t < NB3; t += NT) {
    const int lx = t % NB, ly = (t / NB) % NB, lz = t / (NB * NB);
    if (!(lx < mx && ly < my && lz < mz)) continue;
    T acc[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[f] = T(0);
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
          const int a = i + 4 * j + 16 * k;
#pragma unroll
          for (int f = 0; f < NF; ++f) acc[f] += ev[(slot * NF + f) * 64 + a];
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

// Brick-buffer scatter. The buffer is an extended node grid in which every brick owns
// its own (2P-1)^3 nodes, faces duplicated: brick b's node (lx, ly, lz) sits at
// extended coordinates (NB bx + lx, NB by + ly, NB bz + lz), NB = 2P-1, field-major,
// x fastest. A global x-row of nodes then maps to consecutive extended positions
// (one gap per brick), so both the store and the gather below are coalesced.
__host__ __device__ inline int64_t ext_index(const MeshDev& m, int NB, int f, int gx, int gy, int gz) {
  const int64_t NXe = (int64_t)m.nbx * NB, NYe = (int64_t)m.nby * NB, NZe = (int64_t)m.nbz * NB;
  return ((f * NZe + gz) * NYe + gy) * NXe + gx;
}

// First half: the brick's node sums (same order as scatter_brick4) stored
// unconditionally into the extended grid.
template <typename T, int P, int NF>
__device__ inline void store_brick4(const T* ev, const MeshDev& m, const BrickGeom& g, T* __restrict__ eb) {
  constexpr int p = P - 1, NB = 2 * P - 1, NB3 = NB * NB * NB;
  const int mx = g.nex * p + 1, my = g.ney * p + 1, mz = g.nez * p + 1;
  for (int t = threadIdx.x; t < NB3; t += NT) {
    const int lx = t % NB, ly = (t / NB) % NB, lz = t / (NB * NB);
    if (!(lx < mx && ly < my && lz < mz)) continue;
    T acc[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[f] = T(0);
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
          const int a = i + 4 * j + 16 * k;
#pragma unroll
          for (int f = 0; f < NF; ++f) acc[f] += ev[(slot * NF + f) * 64 + a];
        }
      }
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) eb[ext_index(m, NB, f, NB * g.bx + lx, NB * g.by + ly, NB * g.bz + lz)] = acc[f];
  }
}

// Second half: every node sums the stored values of the (up to 8) blocks holding it
// and stores the result. The buffer is an extended node grid [4][NZe][NYe][NXe] in
// which each block (a brick of 2x2x2 elements, or one element) owns NB nodes per axis
// and the nodes on a face between two blocks appear twice. Along an axis, node i
// (S = NB - 1 nodes per block step) sits at extended position i + i / S of its own
// block, and a node on a block face (i % S == 0, i > 0) also at the position just
// before, in the previous block. One wave per node row (blockIdx.y * 4 + wave,
// blockIdx.z = field); the wave first sums the row's (up to 4) extended rows at every
// extended position (lane = position, so the loads are contiguous), then a face node
// adds the previous position's sum, taken from the neighbouring lane. Lower blocks
// are added first along each axis (deterministic).
template <typename T>
__device__ inline T lane_take(T v, int src);
template <>
__device__ inline double lane_take<double>(double v, int src) {
  return lane_read(v, src);
}
template <>
__device__ inline float lane_take<float>(float v, int src) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}

template <typename T, int NB>
__global__ __launch_bounds__(NT) void k_gather_ext(const T* __restrict__ eb, int nbx, int nby, int nbz, int nx1,
                                                   int ny1, int n_rows, int64_t n_nodes, T* __restrict__ out) {
  constexpr int S = NB - 1;
  const int f = blockIdx.z, w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int NXe = nbx * NB;
  const int64_t NYe = (int64_t)nby * NB, NZe = (int64_t)nbz * NB;
  const T* ebf = eb + f * NZe * NYe * NXe;
  for (int r = blockIdx.y * 4 + w; r < n_rows; r += gridDim.y * 4) {
    const int iz = r / ny1, iy = r - iz * ny1;
    const bool yo = iy / S < nby, yp = iy % S == 0 && iy >= S;
    const bool zo = iz / S < nbz, zp = iz % S == 0 && iz >= S;
    const int64_t gy = iy + iy / S, gz = iz + iz / S;
    // extended rows: own / previous block along z (index 0 / 1) and y (0 / 1)
    const T* rows[4];
    int nr = 0;
    if (zp && yp) rows[nr++] = ebf + ((gz - 1) * NYe + gy - 1) * NXe;
    if (zp && yo) rows[nr++] = ebf + ((gz - 1) * NYe + gy) * NXe;
    if (zo && yp) rows[nr++] = ebf + (gz * NYe + gy - 1) * NXe;
    if (zo && yo) rows[nr++] = ebf + (gz * NYe + gy) * NXe;
    T* orow = out + f * n_nodes + (int64_t)r * nx1;
    for (int j0 = 0; j0 < NXe; j0 += 64) {
      const int j = j0 + l;
      const bool in = j < NXe;
      T sv = T(0);
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (k < nr && in) sv += rows[k][j];
      T prev = lane_take(sv, l > 0 ? l - 1 : 0);
      const int b = j / NB, q = j - b * NB;
      const bool face = q == 0 && j >= NB;
      if (l == 0 && face) {  // the previous position belongs to the previous 64-lane chunk
        prev = T(0);
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (k < nr) prev += rows[k][j - 1];
      }
      if (in) {
        const int ix = j - b;  // node of position j (q < NB - 1)
        if (q < NB - 1) {
          if (ix < nx1) orow[ix] = face ? prev + sv : sv;
        } else if (ix == nx1 - 1) {  // last position of the last block: the row's end node
          orow[ix] = sv;
        }
      }
    }
  }
}

// Global node of lane (x, y, z) of element slot (sx, sy, sz) of the brick; -1 if
// the lane is outside the element's P^3 nodes.
template <int P>
__device__ inline int64_t lane_node(const BrickGeom& g, int sx, int sy, int sz, int nx1, int ny1) {
  const int l = threadIdx.x & 63;
  const int x = l & 3, y = (l >> 2) & 3, z = l >> 4;
  if (x >= P || y >= P || z >= P) return -1;
  constexpr int p = P - 1;
  return (int64_t)((g.ex0 + sx) * p + x) + (int64_t)nx1 * (((g.ey0 + sy) * p + y) + (int64_t)ny1 * ((g.ez0 + sz) * p + z));
}

// Table restriction: global node of lane (x, y, z) of element e, -1 outside its P^3 nodes.
template <int P>
__device__ inline int64_t tab_lane_node(const OpArgs& a, int64_t e) {
  const int l = threadIdx.x & 63;
  const int x = l & 3, y = (l >> 2) & 3, z = l >> 4;
  if (x >= P || y >= P || z >= P) return -1;
  return a.conn[e * (P * P * P) + x + P * (y + P * z)];
}

// FP64 residual / Jacobian / adjoint on Q3 elements with matrix-core sum factorisation.
// GEO: mapped elements, each point's J^-1 and weight read from the geometry record a.qd.
// TAB: table restriction (with GEO): the workgroup takes a group of 8 consecutive elements,
// lane l of an element reads global node a.conn[e * 64 + l], and the element vector goes
// straight to a.evec (summed per node afterwards by k_gather_csr).
template <int MODE, bool BB, bool VOCE, bool MB, bool GEO, bool TAB = false>
__global__ __launch_bounds__(NT, 2) void k_op64_q3(OpArgs a, int colour, DevTables* __restrict__ tabs) {
  static_assert(!TAB || (GEO && !MB), "the table restriction runs on mapped elements without branches");
  __shared__ double ev[8 * 4 * 64];
  __shared__ double red[NT];
  __shared__ double mbs[MB ? 18 * NT : 1];  // branches in parallel: G and W (or Pb) per thread
  const Slot9 sG{mbs + threadIdx.x, NT}, sW{mbs + 9 * NT + threadIdx.x, NT};
  // BB: all bricks in one launch, brick sums to a buffer (see store_brick4); TAB: the
  // workgroup's group of 8 elements
  const int brick = TAB ? xcd_group(a.n_groups, blockIdx.x)
                        : (BB ? xcd_brick_all(a.m, blockIdx.x) : xcd_brick(a.m, colour, blockIdx.x));
  if (brick < 0) return;  // padding workgroup (uniform)
  const BrickGeom g = TAB ? BrickGeom{} : (BB ? decode_brick_lin(a.m, brick) : decode_brick(a.m, colour, brick));
  const Basis4 bs = load_basis4<4>(tabs);
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int qx = l & 3, qz = (l >> 2) & 3, qy = l >> 4;
  const int ql = qx + 4 * qy + 16 * qz;
  const double ih[3] = {a.m.ih[0], a.m.ih[1], a.m.ih[2]};
  const double wbox = tabs->w[4][qx] * tabs->w[4][qy] * tabs->w[4][qz] * a.m.jdet;
  // adjoint: parameter partials and phase id of every point of the brick (slot, lane)
  __shared__ double gpq[MODE == M_ADJ ? 8 * 3 * 64 : 1];
  __shared__ unsigned char gpid[MODE == M_ADJ ? 8 * 64 : 1];
  if (MODE == M_ADJ) {
    gpid[wv * 64 + l] = 255;
    gpid[(wv + 4) * 64 + l] = 255;
  }
  bool any_bad = false, bad_pid = false;
#pragma unroll 1
  for (int half = 0; half < 2; ++half) {
    const int slot = wv + 4 * half;
    const int sx = slot & 1, sy = (slot >> 1) & 1, sz = slot >> 2;
    if (TAB ? (int64_t)brick * 8 + slot >= a.n_elem : !(sx < g.nex && sy < g.ney && sz < g.nez)) continue;  // uniform per wave
    const int64_t e = TAB ? (int64_t)brick * 8 + slot
                          : (int64_t)(g.ex0 + sx) + (int64_t)a.m.nx * ((g.ey0 + sy) + (int64_t)a.m.ny * (g.ez0 + sz));
    const int64_t gn = TAB ? tab_lane_node<4>(a, e) : lane_node<4>(g, sx, sy, sz, a.nx1, a.ny1);
    // gather the element's nodal values (lane = node)
    double zu[4], wu[4], pn = 0.0;
#pragma unroll
    for (int f = 0; f < 4; ++f) zu[f] = a.z[f * a.n_nodes + gn];
    if (MODE != M_RES) {
#pragma unroll
      for (int f = 0; f < 4; ++f) wu[f] = a.w[f * a.n_nodes + gn];
    } else {
      pn = a.phin[gn];
    }
    // per-point state, issued early
    const int64_t gq = e * 64 + ql;
    double st[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) st[k] = a.state[k * a.n_q + gq];
    const int pid = a.phase[gq];
    // mapped elements: the point's J^-1 and weight
    double gA[GEO ? 9 : 1];
    double wdet = wbox;
    if (GEO) {
#pragma unroll
      for (int k = 0; k < 9; ++k) gA[k] = a.qd[k * a.n_q + gq];
      wdet = a.qd[9 * a.n_q + gq];
    }
    // forward sum factorisation
    double G[9], phi = 0.0, gphi[3] = {0.0, 0.0, 0.0}, phin = 0.0;
    {
      double v[4], d[4][3];
      sf4_fwd_n<4>(zu, bs, 0x8u, MODE == M_JAC ? 0x7u : 0xFu, v, d);
#pragma unroll
      for (int f = 0; f < 3; ++f) ref_to_phys<GEO>(d[f], ih, gA, G + 3 * f);
      phi = v[3];
      if (MODE != M_JAC) ref_to_phys<GEO>(d[3], ih, gA, gphi);
    }
    if (MODE == M_RES) {
      double v[1], d[1][3];
      sf4_fwd_n<1>(&pn, bs, 0x1u, 0x0u, v, d);
      phin = v[0];
    }
    // pointwise function (an id outside the phase table raises the phase flag)
    bad_pid |= pid >= a.nph;
    const int pidc = pid < a.nph ? pid : 0;
    const MatParams<double> mp = a.mats[pidc];
    // branches in parallel, adjoint: the extra branches' psi^+ decides the switch
    double psi_x = 0.0;
    if (MB) sG.put(G);
    if (MB && MODE == M_ADJ) psi_x = mb_psi_extra<VOCE>(a, pidc, gq, true, sG, phi, any_bad);
    QPState<double> s;
    qp_state<double, VOCE>(mp, a.fr, G, phi, phin, st, s);
    any_bad |= s.bad;
    // direction (or cotangent) at the points, interpolated after the state so that its
    // 13 values are not live across the state computation
    double W[9], wphi = 0.0, gw[3] = {0.0, 0.0, 0.0};
    if (MODE != M_RES) {
      double v[4], d[4][3];
      sf4_fwd_n<4>(wu, bs, 0x8u, 0xFu, v, d);
#pragma unroll
      for (int f = 0; f < 3; ++f) ref_to_phys<GEO>(d[f], ih, gA, W + 3 * f);
      wphi = v[3];
      ref_to_phys<GEO>(d[3], ih, gA, gw);
    }
    const double kfg = a.fr.kf * mp.Gc;
    double Fu[9], f0, f1[3];
    if (MODE == M_RES) {
      piola<double>(s, Fu);
      double L = s.L;
      if (MB) L = mb_residual<VOCE>(a, mp, pidc, gq, true, sG, phi, phin, st[7], s.psi, s.gp, Fu, any_bad);
#pragma unroll
      for (int k = 0; k < 9; ++k) Fu[k] *= wdet;
      f0 = wdet * a.fr.s_phi * L;
#pragma unroll
      for (int J = 0; J < 3; ++J) f1[J] = wdet * kfg * gphi[J];
    } else if (MODE == M_JAC) {
      double dL;
      if (MB) {
        sW.put(W);
        dL = mb_jacobian<VOCE>(a, mp, s, pidc, gq, true, sG, phi, phi, st[7], W, sW, wphi, Fu, any_bad);
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
      double gsum[3] = {0.0, 0.0, 0.0};
      const double alpha_p = (a.fr.at == 2) ? 2.0 * phi : 1.0;
      gsum[0] += alpha_p * a.fr.inv_c0l0 * Lb + a.fr.kf * wdet * (gphi[0] * gw[0] + gphi[1] * gw[1] + gphi[2] * gw[2]);
      if (s.plastic) {
        const double ee = s.e[0] * s.e[0] + s.e[1] * s.e[1] + s.e[2] * s.e[2];
        const double q = 2.0 * mp.mu * sqrt(1.5 * ee);
        const double w3q = 3.0 * mp.mu / q;
        const double xe = Xd[0] * s.e[0] + Xd[1] * s.e[1] + Xd[2] * s.e[2];
        const double hterm = MB ? Hb * 2.0 * mp.mu * s.c * ee : (s.hactive ? Lb * s.gp * 2.0 * mp.mu * s.c * ee : 0.0);
        const double base = s.g * 2.0 * mp.mu * xe + hterm;
        gsum[1] += -w3q * s.ddg_s0 * base;
        gsum[2] += -w3q * s.ddg_visc * base;
      }
      if (MB) {
        sW.put(Pb);
        mb_adjoint_extra<VOCE>(a, pidc, gq, true, sG, phi, sW, Hb, Fu, phib);
      }
      f0 = phib;
      gpid[slot * 64 + l] = (unsigned char)pid;
#pragma unroll
      for (int k = 0; k < 3; ++k) gpq[(slot * 3 + k) * 64 + l] = gsum[k];
    }
    // backward into the element vector
    {
      double b0[4], b1[4][3], r[4];
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        b0[f] = 0.0;
        phys_to_ref<GEO>(Fu + 3 * f, ih, gA, b1[f]);
      }
      b0[3] = f0;
      phys_to_ref<GEO>(f1, ih, gA, b1[3]);
      sf4_bwd_n<4>(b0, b1, 0x8u, bs, r);
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        if (TAB)
          a.evec[(e * 64 + l) * 4 + f] = r[f];
        else
          ev[(slot * 4 + f) * 64 + l] = r[f];
      }
    }
  }
  if (MODE == M_ADJ) {
    // deterministic per-phase reduction of the parameter partials: a butterfly inside
    // each wave, then the 4 wave sums added in wave order
    // (each thread owns the points (wv, l) and (wv + 4, l), which it wrote itself)
    const int nv = 3 * a.nph;
    const int pid0 = gpid[wv * 64 + l], pid1 = gpid[(wv + 4) * 64 + l];
    if (nv * (NT / 64) <= NT) {
      for (int idx = 0; idx < nv; ++idx) {
        const int ph = idx / 3, k = idx - 3 * ph;
        const double g0 = pid0 == ph ? gpq[(wv * 3 + k) * 64 + l] : 0.0;
        const double g1 = pid1 == ph ? gpq[((wv + 4) * 3 + k) * 64 + l] : 0.0;
        double v = g0 + g1;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (l == 0) red[wv * nv + idx] = v;
      }
      __syncthreads();
      if ((int)threadIdx.x < nv) {
        double t = red[threadIdx.x];
        for (int w = 1; w < NT / 64; ++w) t += red[w * nv + threadIdx.x];
        a.gpart[(int64_t)(a.brick_base + brick) * nv + threadIdx.x] = t;
      }
    } else {
      for (int ph = 0; ph < a.nph; ++ph) {
        for (int k = 0; k < 3; ++k) {
          const double g0 = pid0 == ph ? gpq[(wv * 3 + k) * 64 + l] : 0.0;
          const double g1 = pid1 == ph ? gpq[((wv + 4) * 3 + k) * 64 + l] : 0.0;
          red[threadIdx.x] = g0 + g1;
          __syncthreads();
          for (int st = NT / 2; st > 0; st >>= 1) {
            if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
            __syncthreads();
          }
          if (threadIdx.x == 0) a.gpart[((int64_t)(a.brick_base + brick) * a.nph + ph) * 3 + k] = red[0];
          __syncthreads();
        }
      }
    }
  }
  __syncthreads();
  if (TAB) {
  } else if (BB) {
    store_brick4<double, 4, 4>(ev, a.m, g, a.ebuf);
  } else {
    scatter_brick4<double, 4, 4>(ev, a.m, a.nx1, a.ny1, a.n_nodes, g, a.out);
  }
  if (any_bad) a.flag[0] = 1;
  if (bad_pid) a.flag[1] = 1;
}

}  // namespace pfmf

namespace pfmf {

// FP64 residual / Jacobian / adjoint on Q2 elements (3 nodes, 3 Gauss points per
// direction). Sum factorisation on the matrix cores with the bases zero-padded to
// 4 x 4 (one element per pass, 27 of 64 lanes carry points); the pointwise function
// then runs on a packed layout holding both elements of the wave (lanes 0-26 and
// 32-58), moved there and back by lane permutes, so that it is evaluated once for
// two elements. GEO: mapped elements (J^-1 and weight per point from a.qd). TAB: table
// restriction (with GEO): a group of 8 consecutive elements per workgroup (wave w: elements
// w and w + 4), nodes from a.conn, element vectors straight to a.evec [n_elem][4][27].
template <int MODE, bool BB, bool VOCE, bool MB, bool GEO, bool TAB = false>
__global__ __launch_bounds__(NT, (MB || GEO) ? 2 : 3) void k_op64_q2(OpArgs a, int colour,
                                                                              DevTables* __restrict__ tabs) {
  static_assert(!TAB || (GEO && !MB), "the table restriction runs on mapped elements without branches");
  __shared__ double ev[8 * 4 * 64];
  __shared__ double red[NT];
  __shared__ double mbs[MB ? 18 * NT : 1];  // branches in parallel: G and W (or Pb) per thread
  const Slot9 sG{mbs + threadIdx.x, NT}, sW{mbs + 9 * NT + threadIdx.x, NT};
  // BB: all bricks in one launch, brick sums to a buffer (see store_brick4); TAB: the
  // workgroup's group of 8 elements
  const int brick = TAB ? xcd_group(a.n_groups, blockIdx.x)
                        : (BB ? xcd_brick_all(a.m, blockIdx.x) : xcd_brick(a.m, colour, blockIdx.x));
  if (brick < 0) return;  // padding workgroup (uniform)
  const BrickGeom g = TAB ? BrickGeom{} : (BB ? decode_brick_lin(a.m, brick) : decode_brick(a.m, colour, brick));
  const Basis4 bs = load_basis_pq<3, 3>(tabs);
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // the wave's two elements: slot wv (sz = 0) and slot wv + 4 (sz = 1)
  const int sx = wv & 1, sy = wv >> 1;
  const int64_t e0 = (int64_t)brick * 8 + wv;  // TAB: elements e0 (half 0) and e0 + 4 (half 1)
  const bool hasA = TAB ? e0 < a.n_elem : sx < g.nex && sy < g.ney;  // uniform per wave
  const bool hasB = TAB ? e0 + 4 < a.n_elem : hasA && g.nez > 1;
  // packed layout: lane l holds point q = l & 31 (q < 27) of element E = l >> 5
  const int E = l >> 5, q = l & 31;
  const int cqx = q % 3, cqy = (q / 3) % 3, cqz = q / 9;
  const bool valid = q < 27 && (E == 0 ? hasA : hasB);
  const int src_fwd = cqx + 4 * cqz + 16 * cqy;  // padded point lane (qx, qz, qy) of point q
  // padded point layout of this lane (backward input) and its packed source
  const int pqx = l & 3, pqz = (l >> 2) & 3, pqy = l >> 4;
  const bool pvalid = pqx < 3 && pqy < 3 && pqz < 3;
  const int pq = pqx + 3 * pqy + 9 * pqz;
  const double ih[3] = {a.m.ih[0], a.m.ih[1], a.m.ih[2]};
  const double wbox = tabs->w[3][cqx < 3 ? cqx : 0] * tabs->w[3][cqy] * tabs->w[3][cqz] *
                      a.m.jdet;
  bool any_bad = false, bad_pid = false;
  int pid = 255;
  double gsum[3] = {0.0, 0.0, 0.0};
  if (hasA) {
    // ---- gather and forward interpolation of z (and phi_n), packed into this lane's point
    double G[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double phi = 0.0, gphi[3] = {0.0, 0.0, 0.0}, phin = 0.0;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      if (half == 1 && !hasB) break;  // uniform
      const int64_t gn = TAB ? tab_lane_node<3>(a, e0 + 4 * half) : lane_node<3>(g, sx, sy, half, a.nx1, a.ny1);
      double zu[4];
#pragma unroll
      for (int f = 0; f < 4; ++f) zu[f] = gn >= 0 ? a.z[f * a.n_nodes + gn] : 0.0;
      double v[4], d[4][3];
      sf4_fwd_n<4>(zu, bs, 0x8u, MODE == M_JAC ? 0x7u : 0xFu, v, d);
      const bool mine = E == half;
#pragma unroll
      for (int f = 0; f < 3; ++f)
#pragma unroll
        for (int J = 0; J < 3; ++J) {
          const double r = lane_read(d[f][J], src_fwd);
          if (mine) G[3 * f + J] = GEO ? r : r * ih[J];  // GEO: reference derivatives, mapped below
        }
      const double rp = lane_read(v[3], src_fwd);
      if (mine) phi = rp;
      if (MODE != M_JAC) {
#pragma unroll
        for (int J = 0; J < 3; ++J) {
          const double r = lane_read(d[3][J], src_fwd);
          if (mine) gphi[J] = GEO ? r : r * ih[J];
        }
      }
      if (MODE == M_RES) {
        double pn = gn >= 0 ? a.phin[gn] : 0.0, pv[1], pd[1][3];
        sf4_fwd_n<1>(&pn, bs, 0x1u, 0x0u, pv, pd);
        const double r = lane_read(pv[0], src_fwd);
        if (mine) phin = r;
      }
    }
    // ---- per-point state (packed layout)
    const int64_t e = TAB ? e0 + 4 * E
                          : (int64_t)(g.ex0 + sx) + (int64_t)a.m.nx * ((g.ey0 + sy) + (int64_t)a.m.ny * (g.ez0 + E));
    const int64_t gq = e * 27 + q;
    double st[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) st[k] = valid ? a.state[k * a.n_q + gq] : 0.0;
    pid = valid ? a.phase[gq] : 255;
    // mapped elements: the point's J^-1 and weight; gradients to physical coordinates
    double gA[GEO ? 9 : 1];
    double wdet = wbox;
    if (GEO) {
#pragma unroll
      for (int k = 0; k < 9; ++k) gA[k] = valid ? a.qd[k * a.n_q + gq] : 0.0;
      wdet = valid ? a.qd[9 * a.n_q + gq] : 0.0;
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        const double dr[3] = {G[3 * f], G[3 * f + 1], G[3 * f + 2]};
        ref_to_phys<true>(dr, ih, gA, G + 3 * f);
      }
      const double dp[3] = {gphi[0], gphi[1], gphi[2]};
      ref_to_phys<true>(dp, ih, gA, gphi);
    }
    bad_pid |= valid && pid >= a.nph;
    const int pidc = pid < a.nph ? pid : 0;
    const MatParams<double> mp = a.mats[pidc];
    // branches in parallel (flags of lanes without a point are dropped)
    bool xbad = false;
    double psi_x = 0.0;
    if (MB) sG.put(G);
    if (MB && MODE == M_ADJ) psi_x = mb_psi_extra<VOCE>(a, pidc, gq, valid, sG, phi, xbad);
    QPState<double> s;
    qp_state<double, VOCE>(mp, a.fr, G, phi, phin, st, s);
    any_bad |= valid && s.bad;
    // ---- direction / cotangent at the point
    double W[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double wphi = 0.0, gw[3] = {0.0, 0.0, 0.0};
    if (MODE != M_RES) {
#pragma unroll
      for (int half = 0; half < 2; ++half) {
        if (half == 1 && !hasB) break;
        const int64_t gn = TAB ? tab_lane_node<3>(a, e0 + 4 * half) : lane_node<3>(g, sx, sy, half, a.nx1, a.ny1);
        double wu[4];
#pragma unroll
        for (int f = 0; f < 4; ++f) wu[f] = gn >= 0 ? a.w[f * a.n_nodes + gn] : 0.0;
        double v[4], d[4][3];
        sf4_fwd_n<4>(wu, bs, 0x8u, 0xFu, v, d);
        const bool mine = E == half;
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
          for (int J = 0; J < 3; ++J) {
            const double r = lane_read(d[f][J], src_fwd);
            if (mine) W[3 * f + J] = GEO ? r : r * ih[J];
          }
        const double rp = lane_read(v[3], src_fwd);
        if (mine) wphi = rp;
#pragma unroll
        for (int J = 0; J < 3; ++J) {
          const double r = lane_read(d[3][J], src_fwd);
          if (mine) gw[J] = GEO ? r : r * ih[J];
        }
      }
      if (GEO) {
#pragma unroll
        for (int f = 0; f < 3; ++f) {
          const double dr[3] = {W[3 * f], W[3 * f + 1], W[3 * f + 2]};
          ref_to_phys<true>(dr, ih, gA, W + 3 * f);
        }
        const double dw[3] = {gw[0], gw[1], gw[2]};
        ref_to_phys<true>(dw, ih, gA, gw);
      }
    }
    // ---- pointwise function (packed layout)
    const double kfg = a.fr.kf * mp.Gc;
    double Fu[9], f0, f1[3];
    if (MODE == M_RES) {
      piola<double>(s, Fu);
      double L = s.L;
      if (MB) L = mb_residual<VOCE>(a, mp, pidc, gq, valid, sG, phi, phin, st[7], s.psi, s.gp, Fu, xbad);
#pragma unroll
      for (int k = 0; k < 9; ++k) Fu[k] *= wdet;
      f0 = wdet * a.fr.s_phi * L;
#pragma unroll
      for (int J = 0; J < 3; ++J) f1[J] = wdet * kfg * gphi[J];
    } else if (MODE == M_JAC) {
      double dL;
      if (MB) {
        sW.put(W);
        dL = mb_jacobian<VOCE>(a, mp, s, pidc, gq, valid, sG, phi, phi, st[7], W, sW, wphi, Fu, xbad);
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
        const double qv = 2.0 * mp.mu * sqrt(1.5 * ee);
        const double w3q = 3.0 * mp.mu / qv;
        const double xe = Xd[0] * s.e[0] + Xd[1] * s.e[1] + Xd[2] * s.e[2];
        const double hterm = MB ? Hb * 2.0 * mp.mu * s.c * ee : (s.hactive ? Lb * s.gp * 2.0 * mp.mu * s.c * ee : 0.0);
        const double base = s.g * 2.0 * mp.mu * xe + hterm;
        gsum[1] = -w3q * s.ddg_s0 * base;
        gsum[2] = -w3q * s.ddg_visc * base;
      }
      if (MB) {
        sW.put(Pb);
        mb_adjoint_extra<VOCE>(a, pidc, gq, valid, sG, phi, sW, Hb, Fu, phib);
      }
      f0 = phib;
      if (!valid) gsum[0] = gsum[1] = gsum[2] = 0.0;
    }
    if (MB) any_bad |= valid && xbad;
    // ---- back to the padded layout of each element, transposed interpolation
    double b1p[4][3];
    double b0p[4];
#pragma unroll
    for (int f = 0; f < 3; ++f) phys_to_ref<GEO>(Fu + 3 * f, ih, gA, b1p[f]);
    phys_to_ref<GEO>(f1, ih, gA, b1p[3]);
    b0p[3] = f0;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      if (half == 1 && !hasB) break;
      const int src = pvalid ? 32 * half + pq : l;  // lanes 0..63 only
      double b0[4], b1[4][3], r[4];
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        b0[f] = 0.0;
#pragma unroll
        for (int J = 0; J < 3; ++J) {
          const double v = lane_read(b1p[f][J], src);
          b1[f][J] = pvalid ? v : 0.0;
        }
      }
      {
        const double v = lane_read(b0p[3], src);
        b0[3] = pvalid ? v : 0.0;
      }
      sf4_bwd_n<4>(b0, b1, 0x8u, bs, r);
      const int slot = wv + 4 * half;
      if (TAB) {
        // nodal layout (x, y, z) = lane bits (0-1, 2-3, 4-5); 27 of 64 lanes hold a node
        const int nx_ = l & 3, ny_ = (l >> 2) & 3, nz_ = l >> 4;
        if (nx_ < 3 && ny_ < 3 && nz_ < 3) {
          const int64_t eh = e0 + 4 * half;
#pragma unroll
          for (int f = 0; f < 4; ++f) a.evec[(eh * 27 + nx_ + 3 * ny_ + 9 * nz_) * 4 + f] = r[f];
        }
      } else {
#pragma unroll
        for (int f = 0; f < 4; ++f) ev[(slot * 4 + f) * 64 + l] = r[f];
      }
    }
  }
  if (MODE == M_ADJ) {
    // deterministic per-phase reduction: butterfly inside each wave, wave sums in order
    const int nv = 3 * a.nph;
    if (nv * (NT / 64) <= NT) {
      for (int idx = 0; idx < nv; ++idx) {
        const int ph = idx / 3, k = idx - 3 * ph;
        double v = pid == ph ? (k == 0 ? gsum[0] : (k == 1 ? gsum[1] : gsum[2])) : 0.0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (l == 0) red[wv * nv + idx] = v;
      }
      __syncthreads();
      if ((int)threadIdx.x < nv) {
        double t = red[threadIdx.x];
        for (int w = 1; w < NT / 64; ++w) t += red[w * nv + threadIdx.x];
        a.gpart[(int64_t)(a.brick_base + brick) * nv + threadIdx.x] = t;
      }
    } else {
      for (int ph = 0; ph < a.nph; ++ph) {
        for (int k = 0; k < 3; ++k) {
          red[threadIdx.x] = pid == ph ? (k == 0 ? gsum[0] : (k == 1 ? gsum[1] : gsum[2])) : 0.0;
          __syncthreads();
          for (int st = NT / 2; st > 0; st >>= 1) {
            if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
            __syncthreads();
          }
          if (threadIdx.x == 0) a.gpart[((int64_t)(a.brick_base + brick) * a.nph + ph) * 3 + k] = red[0];
          __syncthreads();
        }
      }
    }
  }
  __syncthreads();
  if (TAB) {
  } else if (BB) {
    store_brick4<double, 3, 4>(ev, a.m, g, a.ebuf);
  } else {
    scatter_brick4<double, 3, 4>(ev, a.m, a.nx1, a.ny1, a.n_nodes, g, a.out);
  }
  if (any_bad) a.flag[0] = 1;
  if (bad_pid) a.flag[1] = 1;
}

}  // namespace pfmf

namespace pfmf {

// FP32 linearised level apply on a Q2 fine mesh (fine kinematics on P = 3 nodes, level
// nodes PC <= 3, 3 Gauss points): the packing of k_op64_q2 (sum factorisation per
// element on the padded 4 x 4 layout, the pointwise JVP once for both elements of the
// wave on lanes 0-26 and 32-58) with the FP32 record path of k_a32_q3.
template <typename V, int PC, bool BB, bool MB, bool GEO = false>
__global__ __launch_bounds__(NT, 2) void k_a32_q2(LinApplyArgs<V> a, int colour, DevTables* __restrict__ tabs) {
  __shared__ V ev[8 * 4 * 64];
  const int brick = BB ? xcd_brick_all(a.m, blockIdx.x) : xcd_brick(a.m, colour, blockIdx.x);
  if (brick < 0) return;  // padding workgroup (uniform)
  const BrickGeom g = BB ? decode_brick_lin(a.m, brick) : decode_brick(a.m, colour, brick);
  const Basis4 bf = load_basis_pq<3, 3>(tabs);
  const Basis4 bc = load_basis_pq<PC, 3>(tabs);
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int sx = wv & 1, sy = wv >> 1;
  const bool hasA = sx < g.nex && sy < g.ney;  // uniform per wave
  const bool hasB = hasA && g.nez > 1;
  const int E = l >> 5, q = l & 31;
  const int cqx = q % 3, cqy = (q / 3) % 3, cqz = q / 9;
  const bool valid = q < 27 && (E == 0 ? hasA : hasB);
  const int src_fwd = cqx + 4 * cqz + 16 * cqy;
  const int pqx = l & 3, pqz = (l >> 2) & 3, pqy = l >> 4;
  const bool pvalid = pqx < 3 && pqy < 3 && pqz < 3;
  const int pq = pqx + 3 * pqy + 9 * pqz;
  const V ih[3] = {(V)a.m.ih[0], (V)a.m.ih[1], (V)a.m.ih[2]};
  const V wbox = (V)(tabs->w[3][cqx < 3 ? cqx : 0] * tabs->w[3][cqy] * tabs->w[3][cqz < 3 ? cqz : 0] *
                             a.m.jdet);
  if (hasA) {
    V G[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    V W[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    V wphi = 0, gw[3] = {0, 0, 0};
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      if (half == 1 && !hasB) break;  // uniform
      const int64_t gf = lane_node<3>(g, sx, sy, half, a.fine.nx1, a.fine.ny1);
      const int64_t gc = lane_node<PC>(g, sx, sy, half, a.lev.nx1, a.lev.ny1);
      double zu[3], wu[4];
#pragma unroll
      for (int f = 0; f < 3; ++f) zu[f] = gf >= 0 ? (double)a.z32[f * a.fine.n_nodes + gf] : 0.0;
#pragma unroll
      for (int f = 0; f < 4; ++f) wu[f] = gc >= 0 ? (double)a.dz[f * a.lev.n_nodes + gc] : 0.0;
      const bool mine = E == half;
      {
        double v[3], d[3][3];
        sf4_fwd_n<3>(zu, bf, 0x0u, 0x7u, v, d);
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
          for (int J = 0; J < 3; ++J) {
            const double r = lane_read(d[f][J], src_fwd);
            if (mine) G[3 * f + J] = GEO ? (V)r : (V)r * ih[J];  // GEO: reference derivatives, mapped below
          }
      }
      {
        double v[4], d[4][3];
        sf4_fwd_n<4>(wu, bc, 0x8u, 0xFu, v, d);
#pragma unroll
        for (int f = 0; f < 3; ++f)
#pragma unroll
          for (int J = 0; J < 3; ++J) {
            const double r = lane_read(d[f][J], src_fwd);
            if (mine) W[3 * f + J] = GEO ? (V)r : (V)r * ih[J];
          }
        const double rp = lane_read(v[3], src_fwd);
        if (mine) wphi = (V)rp;
#pragma unroll
        for (int J = 0; J < 3; ++J) {
          const double r = lane_read(d[3][J], src_fwd);
          if (mine) gw[J] = GEO ? (V)r : (V)r * ih[J];
        }
      }
    }
    // pointwise JVP from the record (packed layout)
    const int64_t e = (int64_t)(g.ex0 + sx) + (int64_t)a.m.nx * ((g.ey0 + sy) + (int64_t)a.m.ny * (g.ez0 + E));
    const int64_t gq = e * 27 + q;
    // mapped elements: the point's J^-1 and weight; gradients to physical coordinates
    double gA[GEO ? 9 : 1];
    V wdet = wbox;
    if (GEO) {
#pragma unroll
      for (int k = 0; k < 9; ++k) gA[k] = valid ? a.qd[k * a.n_q + gq] : 0.0;
      wdet = valid ? (V)a.qd[9 * a.n_q + gq] : V(0);
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        map_grad<V>((double)G[3 * f], (double)G[3 * f + 1], (double)G[3 * f + 2], gA, G + 3 * f);
        map_grad<V>((double)W[3 * f], (double)W[3 * f + 1], (double)W[3 * f + 2], gA, W + 3 * f);
      }
      map_grad<V>((double)gw[0], (double)gw[1], (double)gw[2], gA, gw);
    }
    LinRecordT<V> rc;
#pragma unroll
    for (int k = 0; k < REC_N; ++k) rc.v[k] = valid ? a.rec.rec[k * a.n_q + gq] : V(0);
    rc.flags = valid ? a.rec.flags[gq] : 0;
    const int pid = valid ? a.phase[gq] : 0;
    const int pidc = pid < a.nph ? pid : 0;
    const MatParams<V> mp = a.mats[pidc];
    QPState<V> s;
    qp_state_lin<V>(mp, G, rc, s);
    V Fu[9], dL;
    lin_tangent<V, MB>(a.rec, a.n_q, a.xmats, a.n_extra, mp, s, pidc, gq, valid, G, W, wphi, Fu, dL);
    const V kfg = a.fr.kf * mp.Gc;
    double b1p[4][3], b0p3;
    if (GEO) {
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        double fl[3];
#pragma unroll
        for (int J = 0; J < 3; ++J) fl[J] = f < 3 ? (double)(wdet * Fu[3 * f + J]) : (double)(wdet * kfg * gw[J]);
        phys_to_ref<true>(fl, nullptr, gA, b1p[f]);
      }
    } else {
#pragma unroll
      for (int f = 0; f < 3; ++f)
#pragma unroll
        for (int J = 0; J < 3; ++J) b1p[f][J] = (double)(wdet * Fu[3 * f + J] * ih[J]);
#pragma unroll
      for (int J = 0; J < 3; ++J) b1p[3][J] = (double)(wdet * kfg * gw[J] * ih[J]);
    }
    b0p3 = (double)(wdet * a.fr.s_phi * dL);
    // back to each element's padded layout, transposed interpolation
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      if (half == 1 && !hasB) break;
      const int src = pvalid ? 32 * half + pq : l;
      double b0[4], b1[4][3], r[4];
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        b0[f] = 0.0;
#pragma unroll
        for (int J = 0; J < 3; ++J) {
          const double v = lane_read(b1p[f][J], src);
          b1[f][J] = pvalid ? v : 0.0;
        }
      }
      {
        const double v = lane_read(b0p3, src);
        b0[3] = pvalid ? v : 0.0;
      }
      sf4_bwd_n<4>(b0, b1, 0x8u, bc, r);
      const int slot = wv + 4 * half;
#pragma unroll
      for (int f = 0; f < 4; ++f) ev[(slot * 4 + f) * 64 + l] = (V)r[f];
    }
  }
  __syncthreads();
  if (BB)
    store_brick4<V, PC, 4>(ev, a.m, g, a.ebuf);
  else
    scatter_brick4<V, PC, 4>(ev, a.m, a.lev.nx1, a.lev.ny1, a.lev.n_nodes, g, a.out);
}

// FP32 linearised level apply on a Q3 fine mesh (fine kinematics on P = 4 nodes,
// level nodes PC <= 4, 4 Gauss points): FP32 storage and pointwise arithmetic,
// contractions on the FP64 matrix cores (at the FP32 vector rate on this chip).
template <typename V, int PC, bool BB, bool MB, bool GEO = false>
__global__ __launch_bounds__(NT, 2) void k_a32_q3(LinApplyArgs<V> a, int colour, DevTables* __restrict__ tabs) {
  __shared__ V ev[8 * 4 * 64];
  // BB: all bricks in one launch, brick sums to a buffer (see store_brick4)
  const int brick = BB ? xcd_brick_all(a.m, blockIdx.x) : xcd_brick(a.m, colour, blockIdx.x);
  if (brick < 0) return;  // padding workgroup (uniform)
  const BrickGeom g = BB ? decode_brick_lin(a.m, brick) : decode_brick(a.m, colour, brick);
  const Basis4 bf = load_basis4<4>(tabs);
  const Basis4 bc = load_basis4<PC>(tabs);
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int qx = l & 3, qz = (l >> 2) & 3, qy = l >> 4;
  const int ql = qx + 4 * qy + 16 * qz;
  const V ih[3] = {(V)a.m.ih[0], (V)a.m.ih[1], (V)a.m.ih[2]};
  const V wbox = (V)(tabs->w[4][qx] * tabs->w[4][qy] * tabs->w[4][qz] * a.m.jdet);
#pragma unroll 1
  for (int half = 0; half < 2; ++half) {
    const int slot = wv + 4 * half;
    const int sx = slot & 1, sy = (slot >> 1) & 1, sz = slot >> 2;
    if (!(sx < g.nex && sy < g.ney && sz < g.nez)) continue;  // uniform per wave
    const int64_t gf = lane_node<4>(g, sx, sy, sz, a.fine.nx1, a.fine.ny1);
    const int64_t gc = lane_node<PC>(g, sx, sy, sz, a.lev.nx1, a.lev.ny1);
    double zu[3], wu[4];
#pragma unroll
    for (int f = 0; f < 3; ++f) zu[f] = (double)a.z32[f * a.fine.n_nodes + gf];
#pragma unroll
    for (int f = 0; f < 4; ++f) wu[f] = gc >= 0 ? (double)a.dz[f * a.lev.n_nodes + gc] : 0.0;
    const int64_t e = (int64_t)(g.ex0 + sx) + (int64_t)a.m.nx * ((g.ey0 + sy) + (int64_t)a.m.ny * (g.ez0 + sz));
    const int64_t gq = e * 64 + ql;
    LinRecordT<V> rc;
#pragma unroll
    for (int k = 0; k < REC_N; ++k) rc.v[k] = a.rec.rec[k * a.n_q + gq];
    rc.flags = a.rec.flags[gq];
    const int pid = a.phase[gq];
    // mapped elements: the point's J^-1 and weight
    double gA[GEO ? 9 : 1];
    V wdet = wbox;
    if (GEO) {
#pragma unroll
      for (int k = 0; k < 9; ++k) gA[k] = a.qd[k * a.n_q + gq];
      wdet = (V)a.qd[9 * a.n_q + gq];
    }
    V G[9], W[9], wphi, gw[3];
    {
      double v[3], d[3][3];
      sf4_fwd_n<3>(zu, bf, 0x0u, 0x7u, v, d);
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        if (GEO)
          map_grad<V>(d[f][0], d[f][1], d[f][2], gA, G + 3 * f);
        else
#pragma unroll
          for (int J = 0; J < 3; ++J) G[3 * f + J] = (V)d[f][J] * ih[J];
      }
    }
    {
      double v[4], d[4][3];
      sf4_fwd_n<4>(wu, bc, 0x8u, 0xFu, v, d);
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        if (GEO)
          map_grad<V>(d[f][0], d[f][1], d[f][2], gA, W + 3 * f);
        else
#pragma unroll
          for (int J = 0; J < 3; ++J) W[3 * f + J] = (V)d[f][J] * ih[J];
      }
      wphi = (V)v[3];
      if (GEO)
        map_grad<V>(d[3][0], d[3][1], d[3][2], gA, gw);
      else
#pragma unroll
        for (int J = 0; J < 3; ++J) gw[J] = (V)d[3][J] * ih[J];
    }
    const int pidc = pid < a.nph ? pid : 0;
    const MatParams<V> mp = a.mats[pidc];
    QPState<V> s;
    qp_state_lin<V>(mp, G, rc, s);
    V Fu[9], dL;
    lin_tangent<V, MB>(a.rec, a.n_q, a.xmats, a.n_extra, mp, s, pidc, gq, true, G, W, wphi, Fu, dL);
    const V kfg = a.fr.kf * mp.Gc;
    double b0[4], b1[4][3], r[4];
    if (GEO) {
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        double fl[3];
#pragma unroll
        for (int J = 0; J < 3; ++J) fl[J] = f < 3 ? (double)(wdet * Fu[3 * f + J]) : (double)(wdet * kfg * gw[J]);
        phys_to_ref<true>(fl, nullptr, gA, b1[f]);
        b0[f] = 0.0;
      }
    } else {
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        b0[f] = 0.0;
#pragma unroll
        for (int J = 0; J < 3; ++J) b1[f][J] = (double)(wdet * Fu[3 * f + J] * ih[J]);
      }
#pragma unroll
      for (int J = 0; J < 3; ++J) b1[3][J] = (double)(wdet * kfg * gw[J] * ih[J]);
    }
    b0[3] = (double)(wdet * a.fr.s_phi * dL);
    sf4_bwd_n<4>(b0, b1, 0x8u, bc, r);
#pragma unroll
    for (int f = 0; f < 4; ++f) ev[(slot * 4 + f) * 64 + l] = (V)r[f];
  }
  __syncthreads();
  if (BB)
    store_brick4<V, PC, 4>(ev, a.m, g, a.ebuf);
  else
    scatter_brick4<V, PC, 4>(ev, a.m, a.lev.nx1, a.lev.ny1, a.lev.n_nodes, g, a.out);
}

}  // namespace pfmf
