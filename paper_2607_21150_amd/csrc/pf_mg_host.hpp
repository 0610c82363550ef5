// Host side of the FP32 p-multigrid entry points (included at the end of pfmf.hip).
#pragma once
#include <random>

namespace {

constexpr int VEC_BLOCKS = 2048;

inline int vec_grid(int64_t n) {
  const int64_t b = (n + NT - 1) / NT;
  return (int)(b < VEC_BLOCKS ? (b > 0 ? b : 1) : VEC_BLOCKS);
}

// Nodes of the six boundary faces of a lattice, each face counted in full (k_mask's range).
inline int64_t face_nodes(int nx1, int ny1, int nz1) {
  return 2 * ((int64_t)ny1 * nz1 + (int64_t)nx1 * nz1 + (int64_t)nx1 * ny1);
}

// 1-D transfer rows between orders pf (fine) and pc (coarse) on N elements.
void transfer_rows_1d(int pf, int pc, int N, std::vector<int>& pbase, std::vector<float>& pw,
                      std::vector<int>& rbase, std::vector<float>& rw) {
  std::vector<double> xf, xc, B, D;
  gauss_lobatto(pf + 1, xf);
  gauss_lobatto(pc + 1, xc);
  lagrange_tables(xc, xf, B, D);  // B[il][j] = coarse basis j at fine node il
  const int Pc = pc + 1;
  const int nf = pf * N + 1, nc = pc * N + 1;
  pbase.assign(nf, 0);
  pw.assign((size_t)nf * Pc, 0.f);
  for (int i = 0; i < nf; ++i) {
    const int e = std::min(i / pf, N - 1);
    const int il = i - pf * e;
    pbase[i] = pc * e;
    for (int j = 0; j < Pc; ++j) pw[(size_t)i * Pc + j] = (float)B[il * Pc + j];
  }
  const int nw = 2 * pf + 1;
  rbase.assign(nc, 0);
  rw.assign((size_t)nc * nw, 0.f);
  for (int J = 0; J < nc; ++J) {
    int elo, ehi;
    if (J % pc != 0) {
      elo = ehi = J / pc;
    } else {
      elo = J / pc - 1 < 0 ? 0 : J / pc - 1;
      ehi = J / pc < N ? J / pc : N - 1;
    }
    rbase[J] = pf * elo;
    for (int k = 0; k < nw; ++k) {
      const int i = rbase[J] + k;
      if (i > pf * (ehi + 1) || i >= nf) continue;
      const int e = (i <= pf * (elo + 1)) ? elo : ehi;
      const int il = i - pf * e, j = J - pc * e;
      if (j < 0 || j > pc) continue;
      rw[(size_t)J * nw + k] = (float)B[il * Pc + j];
    }
  }
}

// 1-D transfer rows from an order-1 lattice of Nf (even) elements to the one with Nf / 2:
// fine node i takes coarse node i / 2 (even i, weight 1) or the mean of (i - 1) / 2 and
// (i + 1) / 2 (odd i); restriction is the transpose (weights 1/2, 1, 1/2).
void transfer_rows_h(int Nf, std::vector<int>& pbase, std::vector<float>& pw, std::vector<int>& rbase,
                     std::vector<float>& rw) {
  const int nf = Nf + 1, nc = Nf / 2 + 1;
  pbase.assign(nf, 0);
  pw.assign((size_t)nf * 2, 0.f);
  for (int i = 0; i < nf; ++i) {
    pbase[i] = i / 2;
    if (i % 2 == 0) {
      pw[(size_t)i * 2] = 1.f;
    } else {
      pw[(size_t)i * 2] = 0.5f;
      pw[(size_t)i * 2 + 1] = 0.5f;
    }
  }
  rbase.assign(nc, 0);
  rw.assign((size_t)nc * 3, 0.f);
  for (int J = 0; J < nc; ++J) {
    rbase[J] = 2 * J - 1;
    rw[(size_t)J * 3] = 0.5f;
    rw[(size_t)J * 3 + 1] = 1.f;
    rw[(size_t)J * 3 + 2] = 0.5f;
  }
}

template <typename T>
pf_status upload(T** dst, const std::vector<T>& v) {
  if (hipMalloc(dst, v.size() * sizeof(T)) != hipSuccess) return fail(PF_ENOMEM, "multigrid allocation failed");
  HIPCHK(hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return PF_OK;
}

pf_status mg_alloc_levels(pf_ctx* c, const int* orders, int nl);

pf_status mg_alloc(pf_ctx* c) {
  MGState& mg = c->mg;
  if (mg.n_levels > 0) return PF_OK;
  const int p = c->mesh.p;
  int orders[MG_MAX_LEVELS];
  int nl;
  if (c->n_orders > 0) {
    nl = c->n_orders;
    for (int l = 0; l < c->n_orders; ++l) orders[l] = c->orders[l];
  } else {
    nl = p;
    for (int l = 0; l < p; ++l) orders[l] = p - l;
  }
  // n_levels becomes nl only once every buffer exists; on a failure the partial
  // hierarchy is freed (mg_free) and n_levels stays 0, so a later call starts over
  pf_status st = mg_alloc_levels(c, orders, nl);
  if (st != PF_OK) {
    mg_free(mg);
    return st;
  }
  mg.n_levels = nl;
  return PF_OK;
}

pf_status mg_alloc_levels(pf_ctx* c, const int* orders, int nl) {
  MGState& mg = c->mg;
  const int N[3] = {c->mesh.nx, c->mesh.ny, c->mesh.nz};
  for (int l = 0; l < nl; ++l) {
    MGLevel& L = mg.lv[l];
    L.p = orders[l];
    L.P = L.p + 1;
    // a repeated order 1 coarsens the order-1 lattice by two per direction
    L.h = (l > 0 && L.p == 1 && orders[l - 1] == 1) ? mg.lv[l - 1].h + 1 : 0;
    for (int k = 0; k < 3; ++k) L.ne[k] = L.h > 0 ? mg.lv[l - 1].ne[k] / 2 : N[k];
    L.nx1 = L.p * L.ne[0] + 1;
    L.ny1 = L.p * L.ne[1] + 1;
    L.nz1 = L.p * L.ne[2] + 1;
    L.n_nodes = (int64_t)L.nx1 * L.ny1 * L.nz1;
    const size_t nb = 4 * L.n_nodes * sizeof(float);
    float** bufs[] = {&L.x, &L.r, &L.d, &L.t, &L.b, &L.diag, &L.dinv};
    for (float** b : bufs)
      if (hipMalloc(b, nb) != hipSuccess) return fail(PF_ENOMEM, "multigrid level allocation failed");
    if (L.h > 0 && hipMalloc(&L.S, (size_t)27 * 16 * L.n_nodes * sizeof(float)) != hipSuccess)
      return fail(PF_ENOMEM, "coarse stencil: allocation failed");
    if (l + 1 < nl) {
      const bool hnext = L.p == 1 && orders[l + 1] == 1;
      for (int k = 0; k < 3; ++k) {
        std::vector<int> pb, rb;
        std::vector<float> pw, rw;
        if (hnext)
          transfer_rows_h(L.ne[k], pb, pw, rb, rw);
        else
          transfer_rows_1d(L.p, orders[l + 1], N[k], pb, pw, rb, rw);
        pf_status st;
        if ((st = upload(&L.pbase[k], pb)) || (st = upload(&L.pw[k], pw)) || (st = upload(&L.rbase[k], rb)) ||
            (st = upload(&L.rw[k], rw)))
          return st;
      }
    }
  }
  // the order-1 level on the mesh itself: element matrices and block stencil
  for (int l = 0; l < nl; ++l) {
    if (mg.lv[l].p != 1) continue;
    const int64_t n_elem = (int64_t)c->mesh.nx * c->mesh.ny * c->mesh.nz;
    if (hipMalloc(&mg.ebe, (size_t)n_elem * 1024 * sizeof(float)) != hipSuccess ||
        hipMalloc(&mg.stencil, (size_t)27 * 16 * mg.lv[l].n_nodes * sizeof(float)) != hipSuccess)
      return fail(PF_ENOMEM, "coarse element matrices: allocation failed");
    mg.ebe_level = l;
    break;
  }
  const size_t nfine = 4 * mg.lv[0].n_nodes * sizeof(float);
  if (hipMalloc(&mg.z32, 3 * c->n_nodes * sizeof(float)) != hipSuccess ||
      hipMalloc(&mg.tmpA, nfine) != hipSuccess || hipMalloc(&mg.tmpB, nfine) != hipSuccess ||
      hipMalloc(&mg.red, (VEC_BLOCKS + 16) * sizeof(double)) != hipSuccess)
    return fail(PF_ENOMEM, "multigrid allocation failed");
  return PF_OK;
}

// Record arrays with one layer per branch (the block and the extra branches),
// reallocated when the number of layers changes.
pf_status ensure_records(pf_ctx* c) {
  MGState& mg = c->mg;
  const int layers = 1 + c->n_extra;
  if (mg.rec.rec && mg.rec_layers == layers) return PF_OK;
  (void)hipFree(mg.rec.rec);
  (void)hipFree(mg.rec.flags);
  (void)hipFree(mg.rec64);
  mg.rec = RecordSoA{nullptr, nullptr};
  mg.rec64 = nullptr;
  mg.rec_layers = 0;
  if (hipMalloc(&mg.rec.rec, (size_t)layers * REC_N * c->n_q * sizeof(float)) != hipSuccess ||
      hipMalloc(&mg.rec.flags, (size_t)layers * c->n_q) != hipSuccess)
    return fail(PF_ENOMEM, "linearisation record: allocation failed");
  mg.rec_layers = layers;
  return PF_OK;
}

// Zero the constrained entries of a level vector (no-op without Dirichlet faces).
pf_status mask_level(pf_ctx* c, int level, float* v, hipStream_t s) {
  if (!c->has_dir) return PF_OK;
  const MGLevel& L = c->mg.lv[level];
  hipLaunchKernelGGL(k_mask<float>, dim3(vec_grid(face_nodes(L.nx1, L.ny1, L.nz1))), dim3(NT), 0, s, v, L.nx1, L.ny1, L.nz1, c->dir);
  HIPCHK(hipGetLastError());
  return PF_OK;
}

pf_status mask_fine64(pf_ctx* c, double* v, hipStream_t s) {
  if (!c->has_dir) return PF_OK;
  hipLaunchKernelGGL(k_mask<double>, dim3(vec_grid(face_nodes(c->nx1, c->ny1, c->nz1))), dim3(NT), 0, s, v, c->nx1, c->ny1, c->nz1, c->dir);
  HIPCHK(hipGetLastError());
  return PF_OK;
}

A32Args a32_args(pf_ctx* c, int level, const float* dz, float* out) {
  A32Args a;
  a.m = mesh_dev(c);
  const MGLevel& F = c->mg.lv[0];
  const MGLevel& L = c->mg.lv[level];
  a.fine = LevelDev{F.P, F.nx1, F.ny1, F.n_nodes};
  a.lev = LevelDev{L.P, L.nx1, L.ny1, L.n_nodes};
  a.n_q = c->n_q;
  a.z32 = c->mg.z32;
  a.dz = dz;
  a.rec = c->mg.rec;
  a.phase = c->qp_phase;
  a.mats = c->d_matsf;
  a.nph = (int)c->phases.size();
  a.fr = frac_params<float>(c->fr);
  a.out = out;
  a.ebuf = nullptr;
  a.xmats = c->d_xmatsf;
  a.n_extra = c->n_extra;
  a.qd = c->d_qd32;
  return a;
}

template <int MODE, int PF, int PC, bool MB, bool GEO>
pf_status launch_level32_v(pf_ctx* c, const A32Args& a, hipStream_t s) {
  using S = A32Shape<PF, PC, PF>;
  static bool attr_set = false;
  if (!attr_set) {
    HIPCHK(hipFuncSetAttribute((const void*)k_level32<MODE, PF, PC, PF, MB, GEO>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)S::lds_bytes));
    attr_set = true;
  }
  for (int col = 0; col < 8; ++col) {
    const int nb = xcd_grid(c->nbx, c->nby, c->nbz, col);
    if (nb == 0) continue;
    hipLaunchKernelGGL((k_level32<MODE, PF, PC, PF, MB, GEO>), dim3(nb), dim3(NT), S::lds_bytes, s, a, col, c->d_tabf);
    HIPCHK(hipGetLastError());
  }
  return PF_OK;
}

// kernels with the extra branches' record layers only when branches are attached, with
// the geometry record only on mapped elements (never both: pf_set_geometry checks it)
template <int MODE, int PF, int PC>
pf_status launch_level32(pf_ctx* c, const A32Args& a, hipStream_t s) {
  if (a.qd)
    return a.n_extra > 0 ? launch_level32_v<MODE, PF, PC, true, true>(c, a, s)
                         : launch_level32_v<MODE, PF, PC, false, true>(c, a, s);
  return a.n_extra > 0 ? launch_level32_v<MODE, PF, PC, true, false>(c, a, s)
                       : launch_level32_v<MODE, PF, PC, false, false>(c, a, s);
}

template <int MODE, int PF>
pf_status dispatch_pc(pf_ctx* c, int PC, const A32Args& a, hipStream_t s) {
  switch (PC) {
    case 2: return launch_level32<MODE, PF, 2>(c, a, s);
    case 3: if constexpr (PF >= 3) return launch_level32<MODE, PF, 3>(c, a, s); break;
    case 4: if constexpr (PF >= 4) return launch_level32<MODE, PF, 4>(c, a, s); break;
    case 5: if constexpr (PF >= 5) return launch_level32<MODE, PF, 5>(c, a, s); break;
    default: break;
  }
  return fail(PF_EUNSUPPORTED, "level order not built");
}

// Linearised apply on the matrix cores: PF = 4 (order-3 mesh, k_a32_q3) or PF = 3
// (order-2 mesh, k_a32_q2); V = float for the FP32 levels, V = double for the apply
// from the stored FP64 linearisation (fine level). The brick buffer of each precision
// is sized for the fine level and shared by the coarser ones.
template <typename V, int PF, int PC, bool MB, bool GEO>
pf_status launch_lin_mfma_v(pf_ctx* c, LinApplyArgs<V> a, hipStream_t s) {
  if (use_brick_buffer(c)) {
    V** buf;
    if constexpr (sizeof(V) == 4) buf = &c->mg.ebuf32;
    else buf = &c->d_ebuf;
    constexpr int NBF = 2 * PF - 1;
    if (!*buf && hipMalloc((void**)buf, (size_t)c->n_bricks * 4 * NBF * NBF * NBF * sizeof(V)) != hipSuccess)
      return fail(PF_ENOMEM, "brick buffer: allocation failed");
    a.ebuf = *buf;
    const int ng = xcd_grid_all(c->nbx, c->nby, c->nbz);
    if constexpr (PF == 4) {
      hipLaunchKernelGGL((k_a32_q3<V, PC, true, MB, GEO>), dim3(ng), dim3(NT), 0, s, a, 0, c->d_tab);
    } else if constexpr (!MB && !GEO) {
      // order 2 on box elements without branches: the row-layout kernel (no 3 -> 4 padding)
      if constexpr (sizeof(V) == 4)
        hipLaunchKernelGGL((k_a32_q2r<V, PC>), dim3(ng), dim3(NT), 0, s, a, c->d_tabf);
      else
        hipLaunchKernelGGL((k_a32_q2r<V, PC>), dim3(ng), dim3(NT), 0, s, a, c->d_tab);
    } else {
      hipLaunchKernelGGL((k_a32_q2<V, PC, true, MB, GEO>), dim3(ng), dim3(NT), 0, s, a, 0, c->d_tab);
    }
    HIPCHK(hipGetLastError());
    const int n_rows = (int)(a.lev.n_nodes / a.lev.nx1);
    hipLaunchKernelGGL((k_gather_ext<V, 2 * PC - 1>), dim3(1, std::min((n_rows + 3) / 4, 65535), 4), dim3(NT), 0, s,
                       (const V*)a.ebuf, a.m.nbx, a.m.nby, a.m.nbz, a.lev.nx1, a.lev.ny1, n_rows, a.lev.n_nodes,
                       a.out);
    HIPCHK(hipGetLastError());
    return PF_OK;
  }
  for (int col = 0; col < 8; ++col) {
    const int nb = xcd_grid(c->nbx, c->nby, c->nbz, col);
    if (nb == 0) continue;
    if constexpr (PF == 4)
      hipLaunchKernelGGL((k_a32_q3<V, PC, false, MB, GEO>), dim3(nb), dim3(NT), 0, s, a, col, c->d_tab);
    else
      hipLaunchKernelGGL((k_a32_q2<V, PC, false, MB, GEO>), dim3(nb), dim3(NT), 0, s, a, col, c->d_tab);
    HIPCHK(hipGetLastError());
  }
  return PF_OK;
}

template <typename V, int PF, int PC>
pf_status launch_lin_mfma(pf_ctx* c, const LinApplyArgs<V>& a, hipStream_t s) {
  if (a.qd)
    return a.n_extra > 0 ? launch_lin_mfma_v<V, PF, PC, true, true>(c, a, s)
                         : launch_lin_mfma_v<V, PF, PC, false, true>(c, a, s);
  return a.n_extra > 0 ? launch_lin_mfma_v<V, PF, PC, true, false>(c, a, s)
                       : launch_lin_mfma_v<V, PF, PC, false, false>(c, a, s);
}

template <int PF, int PC>
pf_status launch_a32_mfma(pf_ctx* c, A32Args a, hipStream_t s) {
  return launch_lin_mfma<float, PF, PC>(c, a, s);
}

template <typename V, int PC, bool MB, bool GEO>
pf_status launch_lin_q4_v(pf_ctx* c, const LinApplyArgs<V>& a0, hipStream_t s) {
  LinApplyArgs<V> a = a0;
  if (use_brick_buffer(c)) {
    // element vectors of the level (buffer sized for the fine level), then the node gather
    V** buf;
    if constexpr (sizeof(V) == 4) buf = &c->mg.ebuf32;
    else buf = &c->d_ebuf;
    const int64_t n_elem = (int64_t)c->mesh.nx * c->mesh.ny * c->mesh.nz;
    if (!*buf && hipMalloc((void**)buf, (size_t)n_elem * 4 * 125 * sizeof(V)) != hipSuccess)
      return fail(PF_ENOMEM, "element-vector buffer: allocation failed");
    a.ebuf = *buf;
    const int ng = xcd_grid_elems(c->mesh.nx, c->mesh.ny, c->mesh.nz);
    if constexpr (sizeof(V) == 4)
      hipLaunchKernelGGL((k_a32_q4<V, PC, MB, GEO, true>), dim3(ng), dim3(NT5), 0, s, a, 0, c->d_tabf);
    else
      hipLaunchKernelGGL((k_a32_q4<V, PC, MB, GEO, true>), dim3(ng), dim3(NT5), 0, s, a, 0, c->d_tab);
    HIPCHK(hipGetLastError());
    const int n_rows = (int)(a.lev.n_nodes / a.lev.nx1);
    hipLaunchKernelGGL((k_gather_ext<V, PC>), dim3(1, std::min((n_rows + 3) / 4, 65535), 4), dim3(NT), 0, s,
                       (const V*)a.ebuf, a.m.nx, a.m.ny, a.m.nz, a.lev.nx1, a.lev.ny1, n_rows, a.lev.n_nodes, a.out);
    HIPCHK(hipGetLastError());
    return PF_OK;
  }
  for (int col = 0; col < 8; ++col) {
    const int ng = xcd_grid(c->mesh.nx, c->mesh.ny, c->mesh.nz, col);
    if (ng == 0) continue;
    if constexpr (sizeof(V) == 4)
      hipLaunchKernelGGL((k_a32_q4<V, PC, MB, GEO>), dim3(ng), dim3(NT5), 0, s, a, col, c->d_tabf);
    else
      hipLaunchKernelGGL((k_a32_q4<V, PC, MB, GEO>), dim3(ng), dim3(NT5), 0, s, a, col, c->d_tab);
    HIPCHK(hipGetLastError());
  }
  return PF_OK;
}

template <typename V, int PC>
pf_status launch_lin_q4(pf_ctx* c, const LinApplyArgs<V>& a, hipStream_t s) {
  if (a.qd)
    return a.n_extra > 0 ? launch_lin_q4_v<V, PC, true, true>(c, a, s) : launch_lin_q4_v<V, PC, false, true>(c, a, s);
  return a.n_extra > 0 ? launch_lin_q4_v<V, PC, true, false>(c, a, s) : launch_lin_q4_v<V, PC, false, false>(c, a, s);
}

template <int PC>
pf_status launch_a32_q4(pf_ctx* c, const A32Args& a, hipStream_t s) {
  return launch_lin_q4<float, PC>(c, a, s);
}

EbeArgs ebe_args(pf_ctx* c) {
  EbeArgs a;
  a.m = mesh_dev(c);
  const MGLevel& F = c->mg.lv[0];
  const MGLevel& L = c->mg.lv[c->mg.ebe_level];
  a.fine = LevelDev{F.P, F.nx1, F.ny1, F.n_nodes};
  a.lev = LevelDev{L.P, L.nx1, L.ny1, L.n_nodes};
  a.n_q = c->n_q;
  a.z32 = c->mg.z32;
  a.rec = c->mg.rec;
  a.phase = c->qp_phase;
  a.mats = c->d_matsf;
  a.nph = (int)c->phases.size();
  a.fr = frac_params<float>(c->fr);
  a.K = c->mg.ebe;
  a.xmats = c->d_xmatsf;
  a.n_extra = c->n_extra;
  a.qd = c->d_qd;
  return a;
}

pf_status ebe_assemble(pf_ctx* c, hipStream_t s) {
  const EbeArgs a = ebe_args(c);
  const int n_elem = c->mesh.nx * c->mesh.ny * c->mesh.nz;
  const bool mb = a.n_extra > 0;
  if (a.qd) {  // mapped elements
    switch (c->mg.lv[0].P * 2 + (mb ? 1 : 0)) {
      case 6: hipLaunchKernelGGL((k_ebe_assemble<3, false, true>), dim3(n_elem), dim3(NT), 0, s, a, c->d_tabf); break;
      case 7: hipLaunchKernelGGL((k_ebe_assemble<3, true, true>), dim3(n_elem), dim3(NT), 0, s, a, c->d_tabf); break;
      case 8: hipLaunchKernelGGL((k_ebe_assemble<4, false, true>), dim3(n_elem), dim3(NT), 0, s, a, c->d_tabf); break;
      case 9: hipLaunchKernelGGL((k_ebe_assemble<4, true, true>), dim3(n_elem), dim3(NT), 0, s, a, c->d_tabf); break;
      case 10: hipLaunchKernelGGL((k_ebe_assemble<5, false, true>), dim3(n_elem), dim3(NT), 0, s, a, c->d_tabf); break;
      case 11: hipLaunchKernelGGL((k_ebe_assemble<5, true, true>), dim3(n_elem), dim3(NT), 0, s, a, c->d_tabf); break;
      default: return fail(PF_EUNSUPPORTED, "order not built");
    }
  } else switch (c->mg.lv[0].P * 2 + (mb ? 1 : 0)) {
    case 4: hipLaunchKernelGGL((k_ebe_assemble<2, false>), dim3(n_elem), dim3(NT), 0, s, a, c->d_tabf); break;
    case 5: hipLaunchKernelGGL((k_ebe_assemble<2, true>), dim3(n_elem), dim3(NT), 0, s, a, c->d_tabf); break;
    case 6: hipLaunchKernelGGL((k_ebe_assemble<3, false>), dim3(n_elem), dim3(NT), 0, s, a, c->d_tabf); break;
    case 7: hipLaunchKernelGGL((k_ebe_assemble<3, true>), dim3(n_elem), dim3(NT), 0, s, a, c->d_tabf); break;
    case 8: hipLaunchKernelGGL((k_ebe_assemble<4, false>), dim3(n_elem), dim3(NT), 0, s, a, c->d_tabf); break;
    case 9: hipLaunchKernelGGL((k_ebe_assemble<4, true>), dim3(n_elem), dim3(NT), 0, s, a, c->d_tabf); break;
    case 10: hipLaunchKernelGGL((k_ebe_assemble<5, false>), dim3(n_elem), dim3(NT), 0, s, a, c->d_tabf); break;
    case 11: hipLaunchKernelGGL((k_ebe_assemble<5, true>), dim3(n_elem), dim3(NT), 0, s, a, c->d_tabf); break;
    default: return fail(PF_EUNSUPPORTED, "order not built");
  }
  HIPCHK(hipGetLastError());
  const MGLevel& L = c->mg.lv[c->mg.ebe_level];
  const int64_t nall = 27 * L.n_nodes;
  const int nb = (int)std::min<int64_t>((nall + NT - 1) / NT, 65536);
  hipLaunchKernelGGL(k_stencil_from_ebe, dim3(nb), dim3(NT), 0, s, c->mg.ebe, c->mesh.nx, c->mesh.ny, c->mesh.nz,
                     L.n_nodes, c->mg.stencil);
  HIPCHK(hipGetLastError());
  return PF_OK;
}

// Block-stencil apply (MODE 0) or diagonal (MODE 1) of an order-1 level: the mesh's own
// order-1 level (mg.stencil) or a coarser lattice (its own S).
template <int MODE>
pf_status stencil_apply(pf_ctx* c, int level, const float* x, float* out, hipStream_t s) {
  const MGLevel& L = c->mg.lv[level];
  const float* S = L.h > 0 ? L.S : c->mg.stencil;
  const int nb = (int)std::min<int64_t>((L.n_nodes + NT - 1) / NT, 65536);
  hipLaunchKernelGGL(k_stencil_apply<MODE>, dim3(nb, 4), dim3(NT), 0, s, S, L.nx1, L.ny1, L.nz1, L.n_nodes, x, out);
  HIPCHK(hipGetLastError());
  return PF_OK;
}

template <int MODE>
pf_status ebe_apply(pf_ctx* c, const float* x, float* out, hipStream_t s) {
  return stencil_apply<MODE>(c, c->mg.ebe_level, x, out, s);
}

// Galerkin stencils of the coarser order-1 lattices, each from the level above it.
pf_status build_h_levels(pf_ctx* c, hipStream_t s) {
  MGState& mg = c->mg;
  for (int l = 1; l < mg.n_levels; ++l) {
    const MGLevel& L = mg.lv[l];
    if (L.h == 0) continue;
    const MGLevel& F = mg.lv[l - 1];
    const float* Sf = F.h > 0 ? F.S : mg.stencil;
    const int64_t nall = 27 * 16 * L.n_nodes;
    const int nb = (int)std::min<int64_t>((nall + NT - 1) / NT, 65536);
    hipLaunchKernelGGL(k_stencil_rap, dim3(nb), dim3(NT), 0, s, Sf, F.nx1, F.ny1, F.nz1, L.S, L.nx1, L.ny1, L.nz1);
    HIPCHK(hipGetLastError());
  }
  return PF_OK;
}

template <int MODE>
pf_status level_op_raw(pf_ctx* c, int level, const float* dz, float* out, hipStream_t s) {
  if (c->mg.lv[level].h > 0) return stencil_apply<MODE>(c, level, dz, out, s);
  if (level == c->mg.ebe_level && c->mg.ebe) return ebe_apply<MODE>(c, dz, out, s);
  const A32Args a = a32_args(c, level, dz, out);
  const int PF = c->mg.lv[0].P, PC = c->mg.lv[level].P;
  if (MODE == 0 && PF == 5) {
    switch (PC) {
      case 5: return launch_a32_q4<5>(c, a, s);
      case 4: return launch_a32_q4<4>(c, a, s);
      case 3: return launch_a32_q4<3>(c, a, s);
      case 2: return launch_a32_q4<2>(c, a, s);
      default: break;
    }
  }
  if (MODE == 0 && PF == 4) {
    switch (PC) {
      case 4: return launch_a32_mfma<4, 4>(c, a, s);
      case 3: return launch_a32_mfma<4, 3>(c, a, s);
      case 2: return launch_a32_mfma<4, 2>(c, a, s);
      default: break;
    }
  }
  if (MODE == 0 && PF == 3) {
    switch (PC) {
      case 3: return launch_a32_mfma<3, 3>(c, a, s);
      case 2: return launch_a32_mfma<3, 2>(c, a, s);
      default: break;
    }
  }
  switch (PF) {
    case 2: return dispatch_pc<MODE, 2>(c, PC, a, s);
    case 3: return dispatch_pc<MODE, 3>(c, PC, a, s);
    case 4: return dispatch_pc<MODE, 4>(c, PC, a, s);
    case 5: return dispatch_pc<MODE, 5>(c, PC, a, s);
    default: return fail(PF_EUNSUPPORTED, "order not built");
  }
}

// Level operator; with Dirichlet faces the applied output is masked (M A x), so that
// vectors that vanish on constrained entries stay in that subspace.
template <int MODE>
pf_status level_op(pf_ctx* c, int level, const float* dz, float* out, hipStream_t s) {
  pf_status st = level_op_raw<MODE>(c, level, dz, out, s);
  if (st || MODE != 0) return st;
  return mask_level(c, level, out, s);
}

template <int P, int MODE, bool GEO = false>
pf_status launch_linearize(pf_ctx* c, const LinArgs& a, hipStream_t s) {
  using S = OpShape<P, P>;
  const size_t lds = (4 * S::NB3 + S::TMP + S::TAB) * sizeof(double);
  static bool attr_set = false;
  if (!attr_set) {
    HIPCHK(hipFuncSetAttribute((const void*)k_linearize<P, P, MODE, GEO>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)lds));
    attr_set = true;
  }
  for (int col = 0; col < 8; ++col) {
    const int nb = xcd_grid(c->nbx, c->nby, c->nbz, col);
    if (nb == 0) continue;
    hipLaunchKernelGGL((k_linearize<P, P, MODE, GEO>), dim3(nb), dim3(NT), lds, s, a, col, c->d_tab);
    HIPCHK(hipGetLastError());
  }
  return PF_OK;
}

pf_status sumsq(pf_ctx* c, const float* x, int64_t n, hipStream_t s, double* out) {
  const int g = vec_grid(n);
  hipLaunchKernelGGL(k_sumsq, dim3(g), dim3(NT), 0, s, x, n, c->mg.red);
  HIPCHK(hipGetLastError());
  std::vector<double> h(g);
  HIPCHK(hipMemcpyAsync(h.data(), c->mg.red, g * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  double acc = 0.0;
  for (double v : h) acc += v;
  *out = acc;
  return PF_OK;
}

// y = P x (coarse level l+1 -> level l), separable passes x, y, z.
pf_status prolong(pf_ctx* c, int l, const float* xc, float* xf, hipStream_t s) {
  const MGLevel& F = c->mg.lv[l];
  const MGLevel& C = c->mg.lv[l + 1];
  float* A = c->mg.tmpA;
  float* B = c->mg.tmpB;
  int64_t n;
  n = (int64_t)F.nx1 * C.ny1 * C.nz1;
  hipLaunchKernelGGL(k_transfer_1d, dim3(vec_grid(n)), dim3(NT), 0, s, xc, A, F.nx1, C.ny1, C.nz1, C.nx1, C.ny1,
                     C.nz1, 0, F.pbase[0], F.pw[0], C.P);
  n = (int64_t)F.nx1 * F.ny1 * C.nz1;
  hipLaunchKernelGGL(k_transfer_1d, dim3(vec_grid(n)), dim3(NT), 0, s, A, B, F.nx1, F.ny1, C.nz1, F.nx1, C.ny1,
                     C.nz1, 1, F.pbase[1], F.pw[1], C.P);
  n = F.n_nodes;
  hipLaunchKernelGGL(k_transfer_1d, dim3(vec_grid(n)), dim3(NT), 0, s, B, xf, F.nx1, F.ny1, F.nz1, F.nx1, F.ny1,
                     C.nz1, 2, F.pbase[2], F.pw[2], C.P);
  HIPCHK(hipGetLastError());
  return mask_level(c, l, xf, s);
}

// rc = P^T rf (level l -> coarse level l+1).
pf_status restrict_(pf_ctx* c, int l, const float* rf, float* rc, hipStream_t s) {
  const MGLevel& F = c->mg.lv[l];
  const MGLevel& C = c->mg.lv[l + 1];
  float* A = c->mg.tmpA;
  float* B = c->mg.tmpB;
  const int nw = 2 * F.p + 1;
  int64_t n;
  n = (int64_t)C.nx1 * F.ny1 * F.nz1;
  hipLaunchKernelGGL(k_transfer_1d, dim3(vec_grid(n)), dim3(NT), 0, s, rf, A, C.nx1, F.ny1, F.nz1, F.nx1, F.ny1,
                     F.nz1, 0, F.rbase[0], F.rw[0], nw);
  n = (int64_t)C.nx1 * C.ny1 * F.nz1;
  hipLaunchKernelGGL(k_transfer_1d, dim3(vec_grid(n)), dim3(NT), 0, s, A, B, C.nx1, C.ny1, F.nz1, C.nx1, F.ny1,
                     F.nz1, 1, F.rbase[1], F.rw[1], nw);
  n = C.n_nodes;
  hipLaunchKernelGGL(k_transfer_1d, dim3(vec_grid(n)), dim3(NT), 0, s, B, rc, C.nx1, C.ny1, C.nz1, C.nx1, C.ny1,
                     F.nz1, 2, F.rbase[2], F.rw[2], nw);
  HIPCHK(hipGetLastError());
  return mask_level(c, l + 1, rc, s);
}

// Chebyshev(k) with point Jacobi on level l for A x = b, bounds [0.1, 1.1] * lmax.
pf_status chebyshev(pf_ctx* c, int l, const float* b, float* x, int k, bool x_zero, hipStream_t s) {
  MGLevel& L = c->mg.lv[l];
  const int64_t n = 4 * L.n_nodes;
  const int g = vec_grid(n);
  const double lmax = L.lmax, lmin = 0.1 * L.lmax, lhi = 1.1 * L.lmax;
  const double theta = 0.5 * (lhi + lmin), delta = 0.5 * (lhi - lmin), sigma = theta / delta;
  double rho = 1.0 / sigma;
  (void)lmax;
  pf_status st;
  if (x_zero) {
    hipLaunchKernelGGL(k_vec_copy, dim3(g), dim3(NT), 0, s, b, L.r, n);
  } else {
    if ((st = level_op<0>(c, l, x, L.t, s))) return st;
    hipLaunchKernelGGL(k_vec_sub, dim3(g), dim3(NT), 0, s, b, L.t, L.r, n);
  }
  hipLaunchKernelGGL(k_cheb_first, dim3(g), dim3(NT), 0, s, L.r, L.dinv, L.d, x, (float)(1.0 / theta),
                     x_zero ? 1 : 0, n);
  for (int it = 1; it < k; ++it) {
    if ((st = level_op<0>(c, l, L.d, L.t, s))) return st;
    const double rn = 1.0 / (2.0 * sigma - rho);
    hipLaunchKernelGGL(k_cheb_step, dim3(g), dim3(NT), 0, s, L.r, L.t, L.dinv, L.d, x, (float)(rn * rho),
                       (float)(2.0 * rn / delta), n);
    rho = rn;
  }
  HIPCHK(hipGetLastError());
  return PF_OK;
}

pf_status vcycle(pf_ctx* c, int l, const float* b, float* x, const pf_pmg_opts& o, hipStream_t s) {
  MGState& mg = c->mg;
  MGLevel& L = mg.lv[l];
  const int64_t n = 4 * L.n_nodes;
  const int g = vec_grid(n);
  pf_status st;
  if (l == mg.n_levels - 1) {
    for (int sw = 0; sw < o.coarse_sweeps; ++sw)
      if ((st = chebyshev(c, l, b, x, o.cheb_degree, sw == 0, s))) return st;
    return PF_OK;
  }
  if ((st = chebyshev(c, l, b, x, o.cheb_degree, true, s))) return st;
  if ((st = level_op<0>(c, l, x, L.t, s))) return st;
  hipLaunchKernelGGL(k_vec_sub, dim3(g), dim3(NT), 0, s, b, L.t, L.r, n);
  MGLevel& C = mg.lv[l + 1];
  if ((st = restrict_(c, l, L.r, C.b, s))) return st;
  if ((st = vcycle(c, l + 1, C.b, C.x, o, s))) return st;
  if ((st = prolong(c, l, C.x, L.t, s))) return st;
  hipLaunchKernelGGL(k_vec_add, dim3(g), dim3(NT), 0, s, L.t, x, n);
  HIPCHK(hipGetLastError());
  return chebyshev(c, l, b, x, o.cheb_degree, false, s);
}

pf_status need_lin(pf_ctx* c, int level) {
  pf_status st = check_ctx(c);
  if (st) return st;
  if (!c->mg.linearized) return fail(PF_EINVAL, "call pf_linearize first");
  if (level < 0 || level >= c->mg.n_levels) return fail(PF_EINVAL, "level %d outside 0..%d", level, c->mg.n_levels - 1);
  return PF_OK;
}

}  // namespace

extern "C" {

pf_status pf_linearize(pf_ctx* c, const double* z, void* stream) {
  pf_status st = check_ctx(c);
  if (st) return st;
  if ((st = box_only(c, "pf_linearize"))) return st;
  if (!z) return fail(PF_EINVAL, "null z");
  if (c->n_extra > 0 && c->mesh.p < 2) return fail(PF_EUNSUPPORTED, "extra branches need p >= 2");
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  if ((st = mg_alloc(c)) || (st = ensure_records(c))) return st;
  MGState& mg = c->mg;
  hipLaunchKernelGGL(k_mirror_u, dim3(vec_grid(3 * c->n_nodes)), dim3(NT), 0, s, z, mg.z32, c->n_nodes);
  HIPCHK(hipGetLastError());
  if (c->store_lin64) {
    if ((!mg.rec64 && hipMalloc(&mg.rec64, (size_t)mg.rec_layers * REC_N * c->n_q * sizeof(double)) != hipSuccess) ||
        (!mg.u64 && hipMalloc(&mg.u64, (size_t)3 * c->n_nodes * sizeof(double)) != hipSuccess))
      return fail(PF_ENOMEM, "stored linearisation: allocation failed");
    HIPCHK(hipMemcpyAsync(mg.u64, z, (size_t)3 * c->n_nodes * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  LinArgs a;
  a.m = mesh_dev(c);
  a.nx1 = c->nx1;
  a.ny1 = c->ny1;
  a.n_nodes = c->n_nodes;
  a.n_q = c->n_q;
  a.z = z;
  a.phin = c->phi_n;
  a.state = c->qp_state;
  a.phase = c->qp_phase;
  a.mats = c->d_mats;
  a.nph = (int)c->phases.size();
  a.fr = frac_params<double>(c->fr);
  a.rec = mg.rec;
  a.rec64 = c->store_lin64 ? mg.rec64 : nullptr;
  a.state_out = nullptr;
  a.flag = c->d_flag;
  a.xb = c->d_xb;
  a.xstate = c->xstate;
  a.n_extra = c->n_extra;
  a.xstate_out = nullptr;
  a.qd = c->d_qd;
  const bool mb = c->n_extra > 0;
  if (c->d_qd) {  // mapped elements (orders 2-4: pf_set_geometry checks it)
    switch (c->mesh.p) {
      case 2: st = mb ? launch_linearize<3, 2, true>(c, a, s) : launch_linearize<3, 0, true>(c, a, s); break;
      case 3: st = mb ? launch_linearize<4, 2, true>(c, a, s) : launch_linearize<4, 0, true>(c, a, s); break;
      case 4: st = mb ? launch_linearize<5, 2, true>(c, a, s) : launch_linearize<5, 0, true>(c, a, s); break;
      default: st = fail(PF_EUNSUPPORTED, "order not built");
    }
  } else switch (c->mesh.p) {
    case 1: st = launch_linearize<2, 0>(c, a, s); break;
    case 2: st = mb ? launch_linearize<3, 2>(c, a, s) : launch_linearize<3, 0>(c, a, s); break;
    case 3: st = mb ? launch_linearize<4, 2>(c, a, s) : launch_linearize<4, 0>(c, a, s); break;
    case 4: st = mb ? launch_linearize<5, 2>(c, a, s) : launch_linearize<5, 0>(c, a, s); break;
    default: st = fail(PF_EUNSUPPORTED, "order not built");
  }
  if (st) return st;
  if (mg.ebe_level >= 0 && (st = ebe_assemble(c, s))) return st;
  if ((st = build_h_levels(c, s))) return st;
  mg.linearized = true;
  mg.lin64_valid = c->store_lin64;
  // lambda_max(D^-1 A) per level by 15 power iterations, normalised on the device
  // (no host round trip inside the loop); one synchronisation at the end
  constexpr int POWER_ITS = 15;
  double* nrm = mg.red + VEC_BLOCKS;             // [n_levels] final norms
  float* inv = (float*)(mg.red + VEC_BLOCKS + 8);  // scale of the next normalisation
  for (int l = 0; l < mg.n_levels; ++l) {
    MGLevel& L = mg.lv[l];
    const int64_t n = 4 * L.n_nodes;
    const int g = vec_grid(n);
    if ((st = level_op<1>(c, l, nullptr, L.diag, s))) return st;
    hipLaunchKernelGGL(k_vec_inv, dim3(g), dim3(NT), 0, s, L.diag, L.dinv, n);
    hipLaunchKernelGGL(k_hash_fill, dim3(g), dim3(NT), 0, s, L.d, n, (uint64_t)(21150 + l));
    if ((st = mask_level(c, l, L.d, s))) return st;
    hipLaunchKernelGGL(k_sumsq, dim3(g), dim3(NT), 0, s, L.d, n, mg.red);
    hipLaunchKernelGGL(k_norm_finish, dim3(1), dim3(NT), 0, s, mg.red, g, nrm + l, inv);
    hipLaunchKernelGGL(k_vec_axs_dev, dim3(g), dim3(NT), 0, s, L.d, L.d, inv, n);
    for (int it = 0; it < POWER_ITS; ++it) {
      if ((st = level_op<0>(c, l, L.d, L.t, s))) return st;
      hipLaunchKernelGGL(k_vec_scale, dim3(g), dim3(NT), 0, s, L.dinv, L.t, n);
      hipLaunchKernelGGL(k_sumsq, dim3(g), dim3(NT), 0, s, L.t, n, mg.red);
      hipLaunchKernelGGL(k_norm_finish, dim3(1), dim3(NT), 0, s, mg.red, g, nrm + l, inv);
      hipLaunchKernelGGL(k_vec_axs_dev, dim3(g), dim3(NT), 0, s, L.t, L.d, inv, n);
    }
    HIPCHK(hipGetLastError());
  }
  double lam[MG_MAX_LEVELS];
  HIPCHK(hipMemcpyAsync(lam, nrm, mg.n_levels * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int l = 0; l < mg.n_levels; ++l) {
    if (!(lam[l] > 0.0) || !std::isfinite(lam[l])) return fail(PF_ENONPHYSICAL, "eigenvalue estimate failed on level %d", l);
    mg.lv[l].lmax = lam[l];
  }
  return PF_OK;
}

}  // extern "C"

namespace {

// New per-point state after a converged step (see commit_from_state).
pf_status commit_state(pf_ctx* c, const double* z, double* state_out, double* xstate_out, void* stream) {
  pf_status st = check_ctx(c);
  if (st) return st;
  if ((st = box_only(c, "the state commit"))) return st;
  if (!z || !state_out) return fail(PF_EINVAL, "null argument");
  const size_t ns = 8 * c->n_q * sizeof(double);
  const size_t nz = 4 * c->n_nodes * sizeof(double);
  if (overlaps(state_out, ns, c->qp_state, ns)) return fail(PF_EINVAL, "state_out aliases the context's state");
  if (overlaps(state_out, ns, z, nz)) return fail(PF_EINVAL, "state_out aliases z");
  if (xstate_out) {
    const size_t nx = (size_t)7 * c->n_extra * c->n_q * sizeof(double);
    if (overlaps(xstate_out, nx, c->xstate, nx) || overlaps(xstate_out, nx, c->qp_state, ns) ||
        overlaps(xstate_out, nx, state_out, ns) || overlaps(xstate_out, nx, z, nz))
      return fail(PF_EINVAL, "xstate_out aliases an input or state_out");
  }
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  LinArgs a;
  a.m = mesh_dev(c);
  a.nx1 = c->nx1;
  a.ny1 = c->ny1;
  a.n_nodes = c->n_nodes;
  a.n_q = c->n_q;
  a.z = z;
  a.phin = c->phi_n;
  a.state = c->qp_state;
  a.phase = c->qp_phase;
  a.mats = c->d_mats;
  a.nph = (int)c->phases.size();
  a.fr = frac_params<double>(c->fr);
  a.rec = RecordSoA{nullptr, nullptr};
  a.rec64 = nullptr;
  a.state_out = state_out;
  a.flag = c->d_flag;
  a.xb = c->d_xb;
  a.xstate = c->xstate;
  a.n_extra = c->n_extra;
  a.xstate_out = xstate_out;
  a.qd = c->d_qd;
  const bool mb = c->n_extra > 0;
  if (c->d_qd) {  // mapped elements (orders 2-4: pf_set_geometry checks it)
    switch (c->mesh.p) {
      case 2: return mb ? launch_linearize<3, 3, true>(c, a, s) : launch_linearize<3, 1, true>(c, a, s);
      case 3: return mb ? launch_linearize<4, 3, true>(c, a, s) : launch_linearize<4, 1, true>(c, a, s);
      case 4: return mb ? launch_linearize<5, 3, true>(c, a, s) : launch_linearize<5, 1, true>(c, a, s);
      default: return fail(PF_EUNSUPPORTED, "order not built");
    }
  }
  switch (c->mesh.p) {
    case 1: return launch_linearize<2, 1>(c, a, s);
    case 2: return mb ? launch_linearize<3, 3>(c, a, s) : launch_linearize<3, 1>(c, a, s);
    case 3: return mb ? launch_linearize<4, 3>(c, a, s) : launch_linearize<4, 1>(c, a, s);
    case 4: return mb ? launch_linearize<5, 3>(c, a, s) : launch_linearize<5, 1>(c, a, s);
    default: return fail(PF_EUNSUPPORTED, "order not built");
  }
}

}  // namespace

extern "C" {

pf_status pf_commit_state(pf_ctx* c, const double* z, double* state_out, void* stream) {
  if (c && c->table) return fail(PF_EUNSUPPORTED, "the state commit needs the box lattice");
  if (c && c->n_extra > 0)
    return fail(PF_EUNSUPPORTED, "extra branches attached: use pf_commit_state_branches");
  return commit_state(c, z, state_out, nullptr, stream);
}

pf_status pf_commit_state_branches(pf_ctx* c, const double* z, double* state_out, double* xstate_out,
                                   void* stream) {
  if (c && c->n_extra == 0) return fail(PF_EINVAL, "no extra branch attached: use pf_commit_state");
  if (!xstate_out) return fail(PF_EINVAL, "null xstate_out");
  return commit_state(c, z, state_out, xstate_out, stream);
}

pf_status pf_set_pmg_levels(pf_ctx* c, const int* orders, int n_levels) {
  pf_status st = check_ctx(c);
  if (st) return st;
  if ((st = box_only(c, "pf_set_pmg_levels"))) return st;
  if (n_levels < 0 || n_levels > MG_MAX_LEVELS)
    return fail(PF_EINVAL, "n_levels=%d outside 0..%d", n_levels, MG_MAX_LEVELS);
  if (n_levels > 0 && !orders) return fail(PF_EINVAL, "null orders");
  if (n_levels > 0) {
    if (orders[0] != c->mesh.p) return fail(PF_EINVAL, "the first level must be the mesh order %d", c->mesh.p);
    if (n_levels < 2) return fail(PF_EINVAL, "at least two levels");
    int ne[3] = {c->mesh.nx, c->mesh.ny, c->mesh.nz};
    for (int l = 1; l < n_levels; ++l) {
      if (orders[l] == 1 && orders[l - 1] == 1) {  // a coarser order-1 lattice
        for (int k = 0; k < 3; ++k) {
          if (ne[k] % 2 != 0 || ne[k] < 2)
            return fail(PF_EINVAL, "level %d: an order-1 lattice of %d elements per direction cannot be halved", l,
                        ne[k]);
          ne[k] /= 2;
        }
        continue;
      }
      if (!(orders[l] >= 1 && orders[l] < orders[l - 1]))
        return fail(PF_EINVAL, "orders must decrease to 1, then may repeat 1");
    }
  }
  HIPCHK(hipDeviceSynchronize());
  mg_free(c->mg);
  c->n_orders = n_levels;
  for (int l = 0; l < n_levels; ++l) c->orders[l] = orders[l];
  return PF_OK;
}

pf_status pf_set_dirichlet(pf_ctx* c, const uint32_t* face_fields) {
  pf_status st = check_ctx(c);
  if (st) return st;
  if ((st = box_only(c, "pf_set_dirichlet"))) return st;
  if (!face_fields) return fail(PF_EINVAL, "null face_fields");
  bool any = false;
  for (int k = 0; k < 6; ++k) {
    if (face_fields[k] & ~0xFu) return fail(PF_EINVAL, "face %d: only bits 0..3 (fields) allowed", k);
    c->dir.face[k] = face_fields[k];
    any |= face_fields[k] != 0;
  }
  c->has_dir = any;
  // the diagonals and eigenvalue bounds depend on the mask: linearise again
  c->mg.linearized = false;
  return PF_OK;
}

pf_status pf_level_info(const pf_ctx* c, int level, int* p, int64_t* n_nodes) {
  if (!c) return fail(PF_EINVAL, "null context");
  if (!c->mg.linearized) return fail(PF_EINVAL, "call pf_linearize first");
  if (level < 0 || level >= c->mg.n_levels) return fail(PF_EINVAL, "level %d outside 0..%d", level, c->mg.n_levels - 1);
  if (p) *p = c->mg.lv[level].p;
  if (n_nodes) *n_nodes = c->mg.lv[level].n_nodes;
  return PF_OK;
}

pf_status pf_apply_jacobian_f32(pf_ctx* c, int level, const float* dz, float* y, void* stream) {
  pf_status st = need_lin(c, level);
  if (st) return st;
  if (!dz || !y) return fail(PF_EINVAL, "null vector");
  const size_t nb = 4 * c->mg.lv[level].n_nodes * sizeof(float);
  if (overlaps(dz, nb, y, nb)) return fail(PF_EINVAL, "y aliases dz");
  c->last_stream = (hipStream_t)stream;
  return level_op<0>(c, level, dz, y, (hipStream_t)stream);
}

// FP64 Jacobian at the linearisation point from the stored FP64 record: the FP32
// level apply's kernels instantiated in FP64 on the fine level (u from the copy taken
// at pf_linearize).
pf_status pf_apply_jacobian_lin(pf_ctx* c, const double* dz, double* y, void* stream) {
  pf_status st = check_ctx(c);
  if (st) return st;
  if (!c->mg.linearized || !c->mg.lin64_valid)
    return fail(PF_EINVAL, "call pf_linearize with PF_OPT_STORE_LIN64 on first");
  if (!dz || !y) return fail(PF_EINVAL, "null vector");
  const size_t nb = 4 * c->n_nodes * sizeof(double);
  if (overlaps(dz, nb, y, nb)) return fail(PF_EINVAL, "y aliases dz");
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  LinApplyArgs<double> a;
  a.m = mesh_dev(c);
  const MGLevel& F = c->mg.lv[0];
  a.fine = LevelDev{F.P, F.nx1, F.ny1, F.n_nodes};
  a.lev = a.fine;
  a.n_q = c->n_q;
  a.z32 = c->mg.u64;
  a.dz = dz;
  a.rec = RecordSoAT<double>{c->mg.rec64, c->mg.rec.flags};
  a.phase = c->qp_phase;
  a.mats = c->d_mats;
  a.nph = (int)c->phases.size();
  a.fr = frac_params<double>(c->fr);
  a.out = y;
  a.ebuf = nullptr;
  a.xmats = c->d_xmats64;
  a.n_extra = c->n_extra;
  a.qd = c->d_qd;
  switch (c->mesh.p) {
    case 2: return launch_lin_mfma<double, 3, 3>(c, a, s);
    case 3: return launch_lin_mfma<double, 4, 4>(c, a, s);
    case 4: return launch_lin_q4<double, 5>(c, a, s);
    default: return fail(PF_EUNSUPPORTED, "the stored-linearisation apply is built for orders 2-4");
  }
}

pf_status pf_prolong(pf_ctx* c, int level, const float* xc, float* xf, void* stream) {
  pf_status st = need_lin(c, level);
  if (st) return st;
  if (level + 1 >= c->mg.n_levels) return fail(PF_EINVAL, "no coarser level below %d", level);
  if (!xc || !xf) return fail(PF_EINVAL, "null vector");
  c->last_stream = (hipStream_t)stream;
  return prolong(c, level, xc, xf, (hipStream_t)stream);
}

pf_status pf_restrict(pf_ctx* c, int level, const float* rf, float* rc, void* stream) {
  pf_status st = need_lin(c, level);
  if (st) return st;
  if (level + 1 >= c->mg.n_levels) return fail(PF_EINVAL, "no coarser level below %d", level);
  if (!rf || !rc) return fail(PF_EINVAL, "null vector");
  c->last_stream = (hipStream_t)stream;
  return restrict_(c, level, rf, rc, (hipStream_t)stream);
}

pf_status pf_level_diagonal(pf_ctx* c, int level, float* diag, void* stream) {
  pf_status st = need_lin(c, level);
  if (st) return st;
  if (!diag) return fail(PF_EINVAL, "null vector");
  const int64_t n = 4 * c->mg.lv[level].n_nodes;
  hipLaunchKernelGGL(k_vec_copy, dim3(vec_grid(n)), dim3(NT), 0, (hipStream_t)stream, c->mg.lv[level].diag, diag, n);
  HIPCHK(hipGetLastError());
  return PF_OK;
}

pf_status pf_pmg_vcycle(pf_ctx* c, const float* b, float* x, const pf_pmg_opts* o, void* stream) {
  pf_status st = need_lin(c, 0);
  if (st) return st;
  if (!b || !x) return fail(PF_EINVAL, "null vector");
  const size_t nb = 4 * c->n_nodes * sizeof(float);
  if (overlaps(b, nb, x, nb)) return fail(PF_EINVAL, "x aliases b");
  pf_pmg_opts opt{3, c->mg.lv[c->mg.n_levels - 1].p, 4, 0};
  if (o) {
    if (o->cheb_degree > 0) opt.cheb_degree = o->cheb_degree;
    if (o->coarse_p > 0) opt.coarse_p = o->coarse_p;
    if (o->coarse_sweeps > 0) opt.coarse_sweeps = o->coarse_sweeps;
  }
  if (opt.cheb_degree > 32 || opt.coarse_sweeps > 64) return fail(PF_EINVAL, "smoother degree too large");
  if (opt.coarse_p != c->mg.lv[c->mg.n_levels - 1].p)
    return fail(PF_EINVAL, "coarse_p=%d differs from the coarsest level order %d", opt.coarse_p,
                c->mg.lv[c->mg.n_levels - 1].p);
  c->last_stream = (hipStream_t)stream;
  hipStream_t s = (hipStream_t)stream;
  if (c->has_dir) {
    // work on the masked right-hand side (the V-cycle acts on the unconstrained subspace)
    MGLevel& L = c->mg.lv[0];
    const int64_t n = 4 * L.n_nodes;
    hipLaunchKernelGGL(k_vec_copy, dim3(vec_grid(n)), dim3(NT), 0, s, b, L.b, n);
    if ((st = mask_level(c, 0, L.b, s))) return st;
    return vcycle(c, 0, L.b, x, opt, s);
  }
  return vcycle(c, 0, b, x, opt, s);
}

}  // extern "C"
