// FP64 operator launches (residual, Jacobian, adjoint) for every mesh kind: the generic
// brick kernels (order 1), the matrix-core kernels (orders 2 and 3, brick buffer + gather
// or colour launches, table restriction), the order-4 row-layout kernels.
#pragma once
#include <algorithm>

#include "pf_host.hpp"
#include "pf_mfma.hpp"
#include "pf_q4.hpp"

using namespace pfmf;

template <int MODE, int P, int Q>
pf_status launch_op64(pf_ctx* c, OpArgs a, hipStream_t s) {
  using S = OpShape<P, Q>;
  static bool attr_set = false;
  if (!attr_set) {
    HIPCHK(hipFuncSetAttribute((const void*)k_op64<MODE, P, Q>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)S::lds_bytes));
    attr_set = true;
  }
  for (int col = 0; col < 8; ++col) {
    const int nb = xcd_grid(c->nbx, c->nby, c->nbz, col);
    if (nb == 0) continue;
    a.brick_base = c->colour_base[col];
    hipLaunchKernelGGL((k_op64<MODE, P, Q>), dim3(nb), dim3(NT), S::lds_bytes, s, a, col, c->d_tab);
    HIPCHK(hipGetLastError());
  }
  return PF_OK;
}

template <int MODE, int P, bool VOCE, bool MB, bool GEO>
pf_status launch_op64_mfma_v(pf_ctx* c, OpArgs a, hipStream_t s) {
  const bool bb = use_brick_buffer(c);
  if (bb) {
    constexpr int NB = 2 * P - 1;
    if (!c->d_ebuf &&
        hipMalloc(&c->d_ebuf, (size_t)c->n_bricks * 4 * NB * NB * NB * sizeof(double)) != hipSuccess)
      return fail(PF_ENOMEM, "brick buffer: allocation failed");
    a.ebuf = c->d_ebuf;
    a.brick_base = 0;
    const int ng = xcd_grid_all(c->nbx, c->nby, c->nbz);
    if constexpr (P == 4)
      hipLaunchKernelGGL((k_op64_q3<MODE, true, VOCE, MB, GEO>), dim3(ng), dim3(NT), 0, s, a, 0, c->d_tab);
    else if constexpr (!MB && !GEO)  // box elements without branches: row layout, no 3 -> 4 padding
      hipLaunchKernelGGL((k_op64_q2r<MODE, VOCE>), dim3(ng), dim3(NT), 0, s, a, c->d_tab);
    else
      hipLaunchKernelGGL((k_op64_q2<MODE, true, VOCE, MB, GEO>), dim3(ng), dim3(NT), 0, s, a, 0, c->d_tab);
    HIPCHK(hipGetLastError());
    const int n_rows = c->ny1 * c->nz1;
    hipLaunchKernelGGL((k_gather_ext<double, 2 * P - 1>), dim3(1, std::min((n_rows + 3) / 4, 65535), 4), dim3(NT), 0,
                       s, (const double*)c->d_ebuf, a.m.nbx, a.m.nby, a.m.nbz, c->nx1, c->ny1, n_rows, c->n_nodes,
                       a.out);
    HIPCHK(hipGetLastError());
    return PF_OK;
  }
  for (int col = 0; col < 8; ++col) {
    const int ng = xcd_grid(c->nbx, c->nby, c->nbz, col);
    if (ng == 0) continue;
    a.brick_base = c->colour_base[col];
    if constexpr (P == 4)
      hipLaunchKernelGGL((k_op64_q3<MODE, false, VOCE, MB, GEO>), dim3(ng), dim3(NT), 0, s, a, col, c->d_tab);
    else
      hipLaunchKernelGGL((k_op64_q2<MODE, false, VOCE, MB, GEO>), dim3(ng), dim3(NT), 0, s, a, col, c->d_tab);
    HIPCHK(hipGetLastError());
  }
  return PF_OK;
}

// kernels without the Voce iteration unless a phase uses it; with extra branches
// attached, the branch variant (which carries the Voce iteration for any branch); with
// mapped elements the geometry variant (with or without branches)
template <int MODE, int P>
pf_status launch_op64_mfma(pf_ctx* c, OpArgs a, hipStream_t s) {
  if (c->d_qd && c->n_extra > 0)
    return (c->has_voce || c->xvoce) ? launch_op64_mfma_v<MODE, P, true, true, true>(c, a, s)
                                     : launch_op64_mfma_v<MODE, P, false, true, true>(c, a, s);
  if (c->d_qd)
    return c->has_voce ? launch_op64_mfma_v<MODE, P, true, false, true>(c, a, s)
                       : launch_op64_mfma_v<MODE, P, false, false, true>(c, a, s);
  if (c->n_extra > 0)
    return (c->has_voce || c->xvoce) ? launch_op64_mfma_v<MODE, P, true, true, false>(c, a, s)
                                     : launch_op64_mfma_v<MODE, P, false, true, false>(c, a, s);
  return c->has_voce ? launch_op64_mfma_v<MODE, P, true, false, false>(c, a, s)
                     : launch_op64_mfma_v<MODE, P, false, false, false>(c, a, s);
}

template <int MODE, bool VOCE, bool MB, bool GEO>
pf_status launch_op64_q4_v(pf_ctx* c, OpArgs a, hipStream_t s) {
  if (use_brick_buffer(c)) {
    // element vectors (extended node grid, one block per element) in one launch, then the
    // node gather
    const int64_t n_elem = (int64_t)c->mesh.nx * c->mesh.ny * c->mesh.nz;
    if (!c->d_ebuf && hipMalloc(&c->d_ebuf, (size_t)n_elem * 4 * 125 * sizeof(double)) != hipSuccess)
      return fail(PF_ENOMEM, "element-vector buffer: allocation failed");
    a.evec = c->d_ebuf;
    const int ng = xcd_grid_elems(c->mesh.nx, c->mesh.ny, c->mesh.nz);
    hipLaunchKernelGGL((k_op64_q4<MODE, VOCE, MB, GEO, true>), dim3(ng), dim3(NT5), 0, s, a, 0, c->d_tab);
    HIPCHK(hipGetLastError());
    const int n_rows = c->ny1 * c->nz1;
    hipLaunchKernelGGL((k_gather_ext<double, 5>), dim3(1, std::min((n_rows + 3) / 4, 65535), 4), dim3(NT), 0, s,
                       (const double*)c->d_ebuf, a.m.nx, a.m.ny, a.m.nz, c->nx1, c->ny1, n_rows, c->n_nodes, a.out);
    HIPCHK(hipGetLastError());
    return PF_OK;
  }
  for (int col = 0; col < 8; ++col) {
    const int ng = xcd_grid(c->mesh.nx, c->mesh.ny, c->mesh.nz, col);
    if (ng == 0) continue;
    hipLaunchKernelGGL((k_op64_q4<MODE, VOCE, MB, GEO>), dim3(ng), dim3(NT5), 0, s, a, col, c->d_tab);
    HIPCHK(hipGetLastError());
  }
  return PF_OK;
}

template <int MODE>
pf_status launch_op64_q4(pf_ctx* c, OpArgs a, hipStream_t s) {
  if (c->d_qd && c->n_extra > 0)
    return (c->has_voce || c->xvoce) ? launch_op64_q4_v<MODE, true, true, true>(c, a, s)
                                     : launch_op64_q4_v<MODE, false, true, true>(c, a, s);
  if (c->d_qd)
    return c->has_voce ? launch_op64_q4_v<MODE, true, false, true>(c, a, s)
                       : launch_op64_q4_v<MODE, false, false, true>(c, a, s);
  if (c->n_extra > 0)
    return (c->has_voce || c->xvoce) ? launch_op64_q4_v<MODE, true, true, false>(c, a, s)
                                     : launch_op64_q4_v<MODE, false, true, false>(c, a, s);
  return c->has_voce ? launch_op64_q4_v<MODE, true, false, false>(c, a, s)
                     : launch_op64_q4_v<MODE, false, false, false>(c, a, s);
}

// Table restriction: one launch over the element groups (element vectors to c->d_evec),
// then the node-owner gather into the output.
template <int MODE, int P, bool VOCE>
pf_status launch_op64_tab_v(pf_ctx* c, OpArgs a, hipStream_t s) {
  const int ng = xcd_grid_groups(c->n_groups);
  if constexpr (P == 5)
    hipLaunchKernelGGL((k_op64_q4<MODE, VOCE, false, true, false, true>), dim3(ng), dim3(NT5), 0, s, a, 0, c->d_tab);
  else if constexpr (P == 4)
    hipLaunchKernelGGL((k_op64_q3<MODE, false, VOCE, false, true, true>), dim3(ng), dim3(NT), 0, s, a, 0, c->d_tab);
  else
    hipLaunchKernelGGL((k_op64_q2<MODE, false, VOCE, false, true, true>), dim3(ng), dim3(NT), 0, s, a, 0, c->d_tab);
  HIPCHK(hipGetLastError());
  const int gb = (int)std::min<int64_t>((c->n_nodes + NT - 1) / NT, 1 << 16);
  hipLaunchKernelGGL(k_gather_csr, dim3(gb), dim3(NT), 0, s, (const double*)c->d_evec, (const int32_t*)c->d_csr_off,
                     (const int32_t*)c->d_csr_ent, c->n_nodes, a.out);
  HIPCHK(hipGetLastError());
  return PF_OK;
}

template <int MODE>
pf_status dispatch_op64(pf_ctx* c, OpArgs a, hipStream_t s) {
  if (c->table) {
    if (c->mesh.p == 2)
      return c->has_voce ? launch_op64_tab_v<MODE, 3, true>(c, a, s) : launch_op64_tab_v<MODE, 3, false>(c, a, s);
    if (c->mesh.p == 4)
      return c->has_voce ? launch_op64_tab_v<MODE, 5, true>(c, a, s) : launch_op64_tab_v<MODE, 5, false>(c, a, s);
    return c->has_voce ? launch_op64_tab_v<MODE, 4, true>(c, a, s) : launch_op64_tab_v<MODE, 4, false>(c, a, s);
  }
  switch (c->mesh.p) {
    case 1:
      if (c->n_extra > 0) return fail(PF_EUNSUPPORTED, "extra branches need p >= 2");
      return launch_op64<MODE, 2, 2>(c, a, s);
    case 2: return launch_op64_mfma<MODE, 3>(c, a, s);
    case 3: return launch_op64_mfma<MODE, 4>(c, a, s);
    case 4: return launch_op64_q4<MODE>(c, a, s);
    default: return fail(PF_EUNSUPPORTED, "order p=%d not built", c->mesh.p);
  }
}
