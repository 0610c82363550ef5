// Host side of the FP32 p-multigrid entry points.
#pragma once

extern "C" {

pf_status pf_linearize(pf_ctx* c, const double* z, void* stream) {
  (void)z; (void)stream;
  pf_status st = check_ctx(c);
  if (st) return st;
  return fail(PF_EUNSUPPORTED, "pf_linearize not built");
}

pf_status pf_level_info(const pf_ctx* c, int level, int* p, int64_t* n_nodes) {
  (void)c; (void)level; (void)p; (void)n_nodes;
  return fail(PF_EUNSUPPORTED, "multigrid not built");
}

pf_status pf_apply_jacobian_f32(pf_ctx* c, int level, const float* dz, float* y, void* stream) {
  (void)c; (void)level; (void)dz; (void)y; (void)stream;
  return fail(PF_EUNSUPPORTED, "multigrid not built");
}

pf_status pf_prolong(pf_ctx* c, int level, const float* xc, float* xf, void* stream) {
  (void)c; (void)level; (void)xc; (void)xf; (void)stream;
  return fail(PF_EUNSUPPORTED, "multigrid not built");
}

pf_status pf_restrict(pf_ctx* c, int level, const float* rf, float* rc, void* stream) {
  (void)c; (void)level; (void)rf; (void)rc; (void)stream;
  return fail(PF_EUNSUPPORTED, "multigrid not built");
}

pf_status pf_level_diagonal(pf_ctx* c, int level, float* diag, void* stream) {
  (void)c; (void)level; (void)diag; (void)stream;
  return fail(PF_EUNSUPPORTED, "multigrid not built");
}

pf_status pf_pmg_vcycle(pf_ctx* c, const float* b, float* x, const pf_pmg_opts* o, void* stream) {
  (void)c; (void)b; (void)x; (void)o; (void)stream;
  return fail(PF_EUNSUPPORTED, "multigrid not built");
}

}  // extern "C"
