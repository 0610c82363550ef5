// Host side of the Newton step (included at the end of pfmf.hip): one Newton update
// of the coupled residual with flexible GMRES (right preconditioning, restarted) or,
// on request, preconditioned conjugate gradients, the FP64 Jacobian apply as the
// Krylov operator and one FP32 p-multigrid V-cycle at the FP64 linearisation as the
// preconditioner. Every vector operation runs in
// the kernels of pf_step.hpp; the host holds only the small Hessenberg system.
#pragma once
#include <algorithm>
#include <chrono>

namespace {

// Deterministic dot products <V_j, w>, j = 0..k-1, summed on the host in block order.
pf_status mdot(pf_ctx* c, const double* V, int64_t ld, int k, const double* w, int64_t n, hipStream_t s,
               double* out) {
  const int g = vec_grid(n);
  hipLaunchKernelGGL(k_mdot, dim3(g, k), dim3(NT), 0, s, V, ld, k, w, n, c->kpart);
  HIPCHK(hipGetLastError());
  std::vector<double> h((size_t)g * k);
  HIPCHK(hipMemcpyAsync(h.data(), c->kpart, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int j = 0; j < k; ++j) {
    double acc = 0.0;
    for (int b = 0; b < g; ++b) acc += h[(size_t)j * g + b];
    out[j] = acc;
  }
  return PF_OK;
}

// The k block-partial rows of part summed on the host in block order.
pf_status sum_partials(pf_ctx* c, int g, int k, hipStream_t s, double* out) {
  std::vector<double> h((size_t)g * k);
  HIPCHK(hipMemcpyAsync(h.data(), c->kpart, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int j = 0; j < k; ++j) {
    double acc = 0.0;
    for (int b = 0; b < g; ++b) acc += h[(size_t)j * g + b];
    out[j] = acc;
  }
  return PF_OK;
}

// <V_j, w>, j < k <= GS_MAX, reading w once.
pf_status mdot_multi(pf_ctx* c, const double* V, int64_t ld, int k, const double* w, int64_t n, hipStream_t s,
                     double* out) {
  const int g = vec_grid(n);
  hipLaunchKernelGGL(k_mdot_multi, dim3(g), dim3(NT), 0, s, V, ld, k, w, n, c->kpart);
  HIPCHK(hipGetLastError());
  return sum_partials(c, g, k, s, out);
}

// w += sum_j coef[j] V_j (k <= GS_MAX) and, in the same pass, out = <V_j, w_new> (dots)
// or out[0] = ||w_new||^2.
pf_status gs_correct(pf_ctx* c, const double* V, int64_t ld, int k, const double* coef, double* w, int64_t n,
                     bool dots, hipStream_t s, double* out) {
  HIPCHK(hipMemcpyAsync(c->kcoef, coef, k * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));  // coef is host memory
  const int g = vec_grid(n);
  if (dots)
    hipLaunchKernelGGL(k_maxpy_fused<true>, dim3(g), dim3(NT), 0, s, V, ld, k, c->kcoef, w, n, c->kpart);
  else
    hipLaunchKernelGGL(k_maxpy_fused<false>, dim3(g), dim3(NT), 0, s, V, ld, k, c->kcoef, w, n, c->kpart);
  HIPCHK(hipGetLastError());
  return sum_partials(c, g, dots ? k : 1, s, out);
}

// w += sum_j coef[j] V_j (coef copied from the host, k <= 64)
pf_status maxpy(pf_ctx* c, const double* V, int64_t ld, int k, const double* coef, double* w, int64_t n,
                hipStream_t s) {
  HIPCHK(hipMemcpyAsync(c->kcoef, coef, k * sizeof(double), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));  // coef is host stack memory
  hipLaunchKernelGGL(k_maxpy, dim3(vec_grid(n)), dim3(NT), 0, s, V, ld, k, c->kcoef, w, n);
  HIPCHK(hipGetLastError());
  return PF_OK;
}

pf_status newton_alloc(pf_ctx* c, int m) {
  if (c->kry && c->kry_m >= m) return PF_OK;
  (void)hipFree(c->kry);
  (void)hipFree(c->kpart);
  (void)hipFree(c->kcoef);
  (void)hipFree(c->k32);
  c->kry = nullptr;
  c->kpart = nullptr;
  c->kcoef = nullptr;
  c->k32 = nullptr;
  c->kry_m = 0;
  const int64_t n = 4 * c->n_nodes;
  // V[m+1], Z[m], r, dz, w-spare
  if (hipMalloc(&c->kry, (size_t)(2 * m + 4) * n * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->kpart, (size_t)(m + 2) * VEC_BLOCKS * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->kcoef, 64 * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->k32, (size_t)2 * n * sizeof(float)) != hipSuccess)
    return fail(PF_ENOMEM, "Newton workspace allocation failed (restart %d)", m);
  c->kry_m = m;
  return PF_OK;
}

// x = M^-1 v: FP64 -> FP32, one V-cycle, FP32 -> FP64, masked.
pf_status precondition(pf_ctx* c, const double* v, double* x, const pf_pmg_opts& o, hipStream_t s) {
  const int64_t n = 4 * c->n_nodes;
  const int g = vec_grid(n);
  float* b32 = c->k32;
  float* x32 = c->k32 + n;
  hipLaunchKernelGGL(k_d2f, dim3(g), dim3(NT), 0, s, v, b32, n);
  pf_status st;
  if ((st = mask_level(c, 0, b32, s))) return st;
  if ((st = vcycle(c, 0, b32, x32, o, s))) return st;
  hipLaunchKernelGGL(k_f2d, dim3(g), dim3(NT), 0, s, x32, x, n);
  HIPCHK(hipGetLastError());
  return mask_fine64(c, x, s);
}

// y = M J x on the unconstrained subspace (x vanishes on constrained entries)
// M J(z) x: from the stored FP64 linearisation when the step linearised with it (the
// same operator, without recomputing the point state), else recomputed; with extra
// branches the recompute apply is the faster of the two (the layered FP64 record apply
// spills), so it is used
pf_status masked_jacobian(pf_ctx* c, const double* z, const double* x, double* y, hipStream_t s,
                          bool stored = true) {
  pf_status st;
  if (stored && c->mg.lin64_valid && c->mesh.p >= 2 && c->n_extra == 0) {
    st = pf_apply_jacobian_lin(c, x, y, s);
  } else {
    OpArgs a = op_args(c);
    a.z = z;
    a.w = x;
    a.out = y;
    st = dispatch_op64<M_JAC>(c, a, s);
  }
  if (st) return st;
  return mask_fine64(c, y, s);
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" {

pf_status pf_newton_step(pf_ctx* c, double* z, const pf_newton_opts* o, pf_newton_stats* out, void* stream) {
  pf_status st = check_ctx(c);
  if (st) return st;
  if ((st = box_only(c, "pf_newton_step"))) return st;
  if (!z) return fail(PF_EINVAL, "null z");
  // 32 coarsest-level sweeps: cheap with the element-matrix coarse level, and they
  // cut the FGMRES iterations by 2.5x against 4 sweeps on the Q4 box
  pf_newton_opts opt{1e-8, 30, 300, 3, 32, PF_KRYLOV_FGMRES, {0, 0}};
  if (o) {
    if (o->rtol > 0) opt.rtol = o->rtol;
    if (o->restart > 0) opt.restart = o->restart;
    if (o->max_iters > 0) opt.max_iters = o->max_iters;
    if (o->cheb_degree > 0) opt.cheb_degree = o->cheb_degree;
    if (o->coarse_sweeps > 0) opt.coarse_sweeps = o->coarse_sweeps;
    opt.krylov = o->krylov;
  }
  if (opt.krylov != PF_KRYLOV_FGMRES && opt.krylov != PF_KRYLOV_CG)
    return fail(PF_EINVAL, "krylov %d is neither PF_KRYLOV_FGMRES nor PF_KRYLOV_CG", opt.krylov);
  if (opt.restart > 60) return fail(PF_EINVAL, "restart %d above 60", opt.restart);
  if (opt.cheb_degree > 32 || opt.coarse_sweeps > 64) return fail(PF_EINVAL, "smoother degree too large");
  hipStream_t s = (hipStream_t)stream;
  c->last_stream = s;
  const double t0 = now_ms();
  const int m = std::max(opt.restart, 2);  // CG takes r, p, q from V and its z from Z
  if ((st = newton_alloc(c, m))) return st;
  const int64_t n = 4 * c->n_nodes;
  const int g = vec_grid(n);
  double* V = c->kry;                          // V_j = V + j n, j = 0..m
  double* Z = c->kry + (int64_t)(m + 1) * n;   // Z_j = Z + j n, j = 0..m-1
  double* rhs = Z + (int64_t)m * n;            // b = -M R(z)
  double* dz = rhs + n;                        // accumulated update
  double* w = dz + n;                          // residual of the linear system at restarts
  // right-hand side
  {
    OpArgs a = op_args(c);
    a.z = z;
    a.out = rhs;
    if ((st = dispatch_op64<M_RES>(c, a, s))) return st;
    if ((st = mask_fine64(c, rhs, s))) return st;
    hipLaunchKernelGGL(k_daxpy, dim3(g), dim3(NT), 0, s, -1.0, rhs, rhs, n, 0);
    hipLaunchKernelGGL(k_dzero, dim3(g), dim3(NT), 0, s, dz, n);
    HIPCHK(hipGetLastError());
  }
  double bnorm;
  if ((st = mdot(c, rhs, n, 1, rhs, n, s, &bnorm))) return st;
  bnorm = std::sqrt(bnorm);
  // preconditioner at z
  const double t1 = now_ms();
  if ((st = pf_linearize(c, z, stream))) return st;
  const double t2 = now_ms();
  const pf_pmg_opts po{opt.cheb_degree, c->mg.lv[c->mg.n_levels - 1].p, opt.coarse_sweeps, 0};
  int its = 0, refinements = 0;
  bool conv = bnorm == 0.0, breakdown = false;
  double res = bnorm;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1), h(m + 1), h2(m + 1), y(m);
  if (opt.krylov == PF_KRYLOV_CG && !conv) {
    // preconditioned conjugate gradients on M J dz = b with the same V-cycle. CG assumes a
    // symmetric positive definite operator and preconditioner; the coupled Jacobian is
    // neither in general (s_phi-scaled damage rows, history switch, softening), so the
    // iteration stops at the first p^T J p <= 0 or r^T M r <= 0 (breakdown) or at the limit.
    double* r = V;
    double* p = V + n;
    double* q = V + 2 * n;
    double* zc = Z;
    hipLaunchKernelGGL(k_daxpy, dim3(g), dim3(NT), 0, s, 1.0, rhs, r, n, 0);
    if ((st = precondition(c, r, zc, po, s))) return st;
    hipLaunchKernelGGL(k_daxpy, dim3(g), dim3(NT), 0, s, 1.0, zc, p, n, 0);
    HIPCHK(hipGetLastError());
    double rz;
    if ((st = mdot(c, r, n, 1, zc, n, s, &rz))) return st;
    breakdown = !(rz > 0.0);
    while (!breakdown && its < opt.max_iters) {
      if ((st = masked_jacobian(c, z, p, q, s))) return st;
      double pq;
      if ((st = mdot(c, p, n, 1, q, n, s, &pq))) return st;
      if (!(pq > 0.0)) { breakdown = true; break; }
      const double alpha = rz / pq;
      hipLaunchKernelGGL(k_daxpy, dim3(g), dim3(NT), 0, s, alpha, p, dz, n, 1);
      hipLaunchKernelGGL(k_daxpy, dim3(g), dim3(NT), 0, s, -alpha, q, r, n, 1);
      HIPCHK(hipGetLastError());
      ++its;
      double rr;
      if ((st = mdot(c, r, n, 1, r, n, s, &rr))) return st;
      res = std::sqrt(rr);
      if (res <= opt.rtol * bnorm) { conv = true; break; }
      if ((st = precondition(c, r, zc, po, s))) return st;
      double rz1;
      if ((st = mdot(c, r, n, 1, zc, n, s, &rz1))) return st;
      if (!(rz1 > 0.0)) { breakdown = true; break; }
      const double beta = rz1 / rz;
      rz = rz1;
      hipLaunchKernelGGL(k_daxpy, dim3(g), dim3(NT), 0, s, beta, p, p, n, 0);
      hipLaunchKernelGGL(k_daxpy, dim3(g), dim3(NT), 0, s, 1.0, zc, p, n, 1);
      HIPCHK(hipGetLastError());
    }
  }
  while (opt.krylov == PF_KRYLOV_FGMRES && !conv && its < opt.max_iters) {
    // r = b - J dz (dz = 0 on the first cycle)
    double beta;
    if (its == 0) {
      hipLaunchKernelGGL(k_daxpy, dim3(g), dim3(NT), 0, s, 1.0, rhs, w, n, 0);
    } else {
      if ((st = masked_jacobian(c, z, dz, w, s))) return st;
      hipLaunchKernelGGL(k_daxpy, dim3(g), dim3(NT), 0, s, -1.0, w, w, n, 0);
      hipLaunchKernelGGL(k_daxpy, dim3(g), dim3(NT), 0, s, 1.0, rhs, w, n, 1);
    }
    if ((st = mdot(c, w, n, 1, w, n, s, &beta))) return st;
    beta = std::sqrt(beta);
    res = beta;
    if (beta <= opt.rtol * bnorm) { conv = true; break; }
    hipLaunchKernelGGL(k_daxpy, dim3(g), dim3(NT), 0, s, 1.0 / beta, w, V, n, 0);
    std::fill(gv.begin(), gv.end(), 0.0);
    gv[0] = beta;
    int k = 0;
    for (; k < opt.restart && its < opt.max_iters; ++k, ++its) {
      double* Vk = V + (int64_t)k * n;
      double* Zk = Z + (int64_t)k * n;
      double* Vn = V + (int64_t)(k + 1) * n;
      if ((st = precondition(c, Vk, Zk, po, s))) return st;
      if ((st = masked_jacobian(c, z, Zk, Vn, s))) return st;
      // classical Gram-Schmidt with adaptive refinement (the GMRES variant of Section 5):
      // the first pass also returns ||w||^2 (Vn follows V_k in memory); a second pass runs
      // only when the first removed more than half of it, ||w1||^2 = ||w||^2 - sum h_j^2
      // < ||w||^2 / 2, the point where orthogonality can be lost. With k + 2 <= GS_MAX
      // every pass reads the basis once: the projections read w once, and each correction
      // also yields the next pass's projections (refinement) or the new norm.
      const bool fused = k + 2 <= GS_MAX;
      if ((st = fused ? mdot_multi(c, V, n, k + 2, Vn, n, s, h.data()) : mdot(c, V, n, k + 2, Vn, n, s, h.data())))
        return st;
      const double w0 = h[k + 1];
      double proj = 0.0;
      for (int j = 0; j <= k; ++j) {
        y[j] = -h[j];
        proj += h[j] * h[j];
      }
      const bool refine = !(w0 - proj > 0.5 * w0);
      double hn;
      if (fused) {
        if (refine) {
          ++refinements;
          if ((st = gs_correct(c, V, n, k + 1, y.data(), Vn, n, true, s, h2.data()))) return st;
          for (int j = 0; j <= k; ++j) {
            y[j] = -h2[j];
            h[j] += h2[j];
          }
        }
        if ((st = gs_correct(c, V, n, k + 1, y.data(), Vn, n, false, s, &hn))) return st;
      } else {
        if ((st = maxpy(c, V, n, k + 1, y.data(), Vn, n, s))) return st;
        if (refine) {
          ++refinements;
          if ((st = mdot(c, V, n, k + 1, Vn, n, s, h2.data()))) return st;
          for (int j = 0; j <= k; ++j) {
            y[j] = -h2[j];
            h[j] += h2[j];
          }
          if ((st = maxpy(c, V, n, k + 1, y.data(), Vn, n, s))) return st;
        }
        if ((st = mdot(c, Vn, n, 1, Vn, n, s, &hn))) return st;
      }
      hn = std::sqrt(hn);
      h[k + 1] = hn;
      if (hn > 0.0) hipLaunchKernelGGL(k_daxpy, dim3(g), dim3(NT), 0, s, 1.0 / hn, Vn, Vn, n, 0);
      // Givens rotations on the new column
      for (int j = 0; j < k; ++j) {
        const double t = cs[j] * h[j] + sn[j] * h[j + 1];
        h[j + 1] = -sn[j] * h[j] + cs[j] * h[j + 1];
        h[j] = t;
      }
      const double r = std::hypot(h[k], h[k + 1]);
      cs[k] = r > 0.0 ? h[k] / r : 1.0;
      sn[k] = r > 0.0 ? h[k + 1] / r : 0.0;
      h[k] = r;
      h[k + 1] = 0.0;
      gv[k + 1] = -sn[k] * gv[k];
      gv[k] = cs[k] * gv[k];
      for (int j = 0; j <= k; ++j) H[(size_t)j * m + k] = h[j];
      res = std::fabs(gv[k + 1]);
      if (res <= opt.rtol * bnorm || hn == 0.0) {
        ++k;
        ++its;
        conv = true;
        break;
      }
    }
    // y = R^-1 g, dz += Z y
    for (int i = k - 1; i >= 0; --i) {
      double acc = gv[i];
      for (int j = i + 1; j < k; ++j) acc -= H[(size_t)i * m + j] * y[j];
      y[i] = acc / H[(size_t)i * m + i];
    }
    if ((st = maxpy(c, Z, n, k, y.data(), dz, n, s))) return st;
  }
  // true linear residual ||b - M J dz|| / ||b|| with the recomputed Jacobian (an
  // independent check of the stored one used by the iteration), then z += dz
  if ((st = masked_jacobian(c, z, dz, w, s, false))) return st;
  hipLaunchKernelGGL(k_daxpy, dim3(g), dim3(NT), 0, s, -1.0, w, w, n, 0);
  hipLaunchKernelGGL(k_daxpy, dim3(g), dim3(NT), 0, s, 1.0, rhs, w, n, 1);
  double rt;
  if ((st = mdot(c, w, n, 1, w, n, s, &rt))) return st;
  hipLaunchKernelGGL(k_daxpy, dim3(g), dim3(NT), 0, s, 1.0, dz, z, n, 1);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  const double t3 = now_ms();
  if (out) {
    out->iterations = its;
    out->converged = conv ? 1 : 0;
    out->res0 = bnorm;
    out->res_lin = res;
    out->res_true = std::sqrt(rt);
    out->t_linearize_ms = t2 - t1;
    out->t_total_ms = t3 - t0;
    out->refinements = refinements;
    out->krylov = opt.krylov;
    out->breakdown = breakdown ? 1 : 0;
  }
  return conv ? PF_OK : fail(PF_ENOCONV, "%s did not reach rtol %.1e in %d iterations (%.3e%s)",
                             opt.krylov == PF_KRYLOV_CG ? "CG" : "FGMRES", opt.rtol, its,
                             bnorm > 0 ? res / bnorm : 0.0, breakdown ? ", breakdown" : "");
}

}  // extern "C"
