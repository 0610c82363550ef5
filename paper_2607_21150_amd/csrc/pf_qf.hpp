// Pointwise (quadrature-point) functions of the coupled operator, device side.
//
// Material model (Sections 2-3 of the paper): finite-strain Hencky material,
// Peric-Dettmer block with a Hooke branch or one Prandtl branch (Box 1, Box 2)
// whose yield stress carries linear hardening and an overstress factor
// (1 + a dgamma), a = visc/dt, in series with the phase-field fracture element
// (degradation g = (1-phi)^2 + eta, Amor split, Miehe history, AT1/AT2 crack
// density, damage viscosity). The Prandtl update uses the degraded trial stress
// g*q_tr and g*mu (eq:degraded-trial-stress, eq:degraded-yield-condition).
//
// Everything is formulated in the principal frame of b_tr (Appendix A): the
// stress update acts on eigenvalues, and the tangent (Appendices B-C) acts on
// the rotated perturbation N^T db N, whose off-diagonal part is scaled by the
// divided difference (tau_i - tau_j)/(b_i - b_j) = g mu c (ln b_i - ln b_j)/(b_i - b_j),
// the form of the eigenvector-derivative term that stays finite for equal
// eigenvalues. The inelastic state is carried as D = Cin^-1 - I so that
// A = b_tr - I = G + G^T + G G^T + F D F^T is formed without cancellation.
#pragma once
#include <hip/hip_runtime.h>

namespace pfmf {

template <typename T> struct MatParams {
  T mu, kappa, Gc, sigma0, H, a;  // a = visc / dt
  int plastic;
  T sinf, bv;                     // Voce saturation stress and rate (bv = 0: linear hardening)
  T am;                           // Maxwell branch: mu dt / eta_d (0 for other branches)
};

// Yield stress and its slope at accumulated plastic strain ep
// (eq:plasticity-strain-hardening-law): sigma0 + H ep + (sinf - sigma0)(1 - exp(-bv ep)).
template <typename T>
__device__ inline T yield_stress(const MatParams<T>& m, T ep) {
  return m.sigma0 + m.H * ep + (m.bv > T(0) ? (m.sinf - m.sigma0) * (T(1) - exp(-m.bv * ep)) : T(0));
}
template <typename T>
__device__ inline T yield_slope(const MatParams<T>& m, T ep) {
  return m.H + (m.bv > T(0) ? (m.sinf - m.sigma0) * m.bv * exp(-m.bv * ep) : T(0));
}

template <typename T> struct FracParams {
  T l0, eta, zeta, inv_dt, s_phi, c0, inv_c0l0, kf;  // kf = s_phi * 2 l0 / c0 (times Gc at use)
  int at;
};

__device__ inline double pf_rsqrt(double x) { return rsqrt(x); }
__device__ inline float pf_rsqrt(float x) { return rsqrtf(x); }
__device__ inline double pf_sqrt(double x) { return sqrt(x); }
__device__ inline float pf_sqrt(float x) { return sqrtf(x); }
__device__ inline double pf_log1p(double x) { return log1p(x); }
__device__ inline float pf_log1p(float x) { return log1pf(x); }
__device__ inline double pf_abs(double x) { return fabs(x); }
__device__ inline float pf_abs(float x) { return fabsf(x); }

// Reciprocal and reciprocal square root from the hardware estimate refined by
// two Newton steps (FP64) or used as is (FP32, about 1 ulp). Arguments here are
// finite and positive (or nonzero for the reciprocal) by construction.
__device__ inline double frcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ inline float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double frsqrt(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  double t = fma(-h * y, y, 0.5);
  y = fma(y, t, y);
  t = fma(-h * y, y, 0.5);
  return fma(y, t, y);
}
__device__ inline float frsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
// exp for the FP32 record path: the hardware 2^x with a scaled argument (a few ulp)
__device__ inline double fexp(double x) { return exp(x); }
__device__ inline float fexp(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }

template <typename T> struct Eps;
template <> struct Eps<double> {
  static constexpr double conv = 1e-30;    // squared relative off-diagonal threshold
  static constexpr double tiny = 1e-280;   // below this the 2x2 block is left unrotated
  static constexpr double series = 0.25;   // |x| up to which log1p uses the atanh series
  static constexpr int nterms = 11;        // atanh series terms (relative error < 1e-17)
  static constexpr int max_sweeps = 8;
};
template <> struct Eps<float> {
  static constexpr float conv = 1e-13f;
  static constexpr float tiny = 1e-30f;
  static constexpr float series = 0.25f;
  static constexpr int nterms = 5;
  static constexpr int max_sweeps = 6;
};

// 1 + s^2/3 + s^4/5 + ... (atanh(s)/s), Horner in s^2
// (6 terms when s2 <= 1e-3: the truncation is then below s2^6 / 13 < 1e-19)
template <typename T>
__device__ inline T atanh_ratio(T s2) {
  if (Eps<T>::nterms > 6 && s2 <= T(1e-3)) {
    T r = T(1) / T(11);
#pragma unroll
    for (int k = 4; k >= 0; --k) r = fma(r, s2, T(1) / T(2 * k + 1));
    return r;
  }
  T r = T(1) / T(2 * Eps<T>::nterms - 1);
#pragma unroll
  for (int k = Eps<T>::nterms - 2; k >= 0; --k) r = fma(r, s2, T(1) / T(2 * k + 1));
  return r;
}

// 0.5 log1p(x) = atanh(x / (2 + x)); series for |x| <= 0.25, library beyond.
template <typename T>
__device__ inline T half_log1p(T x) {
  T r;
  if (pf_abs(x) <= Eps<T>::series) {
    const T sv = x * frcp(T(2) + x);
    r = sv * atanh_ratio(sv * sv);
  } else {
    r = T(0.5) * pf_log1p(x);
  }
  return r;
}

// Symmetric 3x3 stored as s[6] = {xx, yy, zz, yz, xz, xy}.
// General 3x3 stored row-major m[9].

// Cyclic Jacobi on a symmetric 3x3: a (overwritten, diagonal on exit holds the
// eigenvalues) and eigenvector matrix V (columns). Uniform sweep count with an
// early exit when the off-diagonal part is negligible.
template <typename T>
__device__ inline void jacobi_rotate(T& app, T& aqq, T& apq, T& arp, T& arq, T* V, int p, int q) {
  // rotation angle phi with tan(2 phi) = 2 apq / (aqq - app), |phi| <= pi/4, from
  // cos(2 phi) = |d|/r, sin(2 phi) = sgn(d) 2 apq / r and the half-angle formulas
  const T d = aqq - app;
  const T o = apq;
  const T r2 = d * d + T(4) * o * o;
  const bool flat = !(r2 > Eps<T>::tiny);
  const T ir = frsqrt(flat ? T(1) : r2);
  const T cos2 = flat ? T(1) : pf_abs(d) * ir;
  const T sin2 = flat ? T(0) : ((d < T(0)) ? T(-2) : T(2)) * o * ir;
  const T h = T(0.5) + T(0.5) * cos2;
  const T ic = frsqrt(h);  // 1 / cos(phi)
  const T c = h * ic;
  const T sn = T(0.5) * sin2 * ic;
  const T t = sn * ic;     // tan(phi)
  app -= t * o;
  aqq += t * o;
  apq = T(0);
  const T rp = c * arp - sn * arq;
  const T rq = sn * arp + c * arq;
  arp = rp;
  arq = rq;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const T vp = V[3 * k + p], vq = V[3 * k + q];
    V[3 * k + p] = c * vp - sn * vq;
    V[3 * k + q] = sn * vp + c * vq;
  }
}

// Seed of c = cos(acos(r) / 3) for r in [-1, 1]. With t = sqrt((1 + r) / 2) =
// cos(acos(r) / 2), c = cos(2 acos(t) / 3) is analytic in t on [0, 1]; it is taken
// as 0.5 + t q(t) with q a degree-7 least-squares Chebyshev-node fit of (c - 0.5) / t
// (exact at r = -1, error below 4e-8 with t from the FP32 square root).
template <typename T>
__device__ inline T seed_cos_third(T r) {
  const float tf = __builtin_sqrtf((float)(T(0.5) * (T(1) + r)));
  const T t = (T)tf;
  T q = T(-0.0008711068611442343);
  q = fma(q, t, T(0.004603595835898712));
  q = fma(q, t, T(-0.011722732125447858));
  q = fma(q, t, T(0.020800135207323198));
  q = fma(q, t, T(-0.03245631158654394));
  q = fma(q, t, T(0.05340486896259051));
  q = fma(q, t, T(-0.11110871404718346));
  q = fma(q, t, T(0.5773502512952833));
  return fma(t, q, T(0.5));
}

// Symmetric 3x3 eigen-decomposition A = V diag(lam) V^T (eigenvectors in the
// columns of V). Closed-form eigenvalues of the deviator (cos(acos(r)/3), seeded
// in FP32 and refined by one Newton step on 4 c^3 - 3 c = r), the null vector of
// A - lam I for the most isolated eigenvalue by cross products, any orthonormal
// completion of it, and one cyclic Jacobi sweep on V^T A V. The sweep removes the
// error of the closed form (second order after one sweep) and diagonalises a
// nearly repeated pair exactly, where the closed form alone is inaccurate.
template <typename T>
__device__ inline void eig_sym3(const T* A, T* lam, T* V) {
  const T a00 = A[0], a11 = A[1], a22 = A[2], a12 = A[3], a02 = A[4], a01 = A[5];
  const T m = (a00 + a11 + a22) * (T(1) / T(3));
  const T s00 = a00 - m, s11 = a11 - m, s22 = a22 - m;
  const T J2 = T(0.5) * (s00 * s00 + s11 * s11 + s22 * s22) + a01 * a01 + a02 * a02 + a12 * a12;
#pragma unroll
  for (int k = 0; k < 9; ++k) V[k] = (k % 4 == 0) ? T(1) : T(0);
  if (J2 > Eps<T>::tiny + Eps<T>::conv * m * m) {
    const T J3 = s00 * (s11 * s22 - a12 * a12) - a01 * (a01 * s22 - a12 * a02) + a02 * (a01 * a12 - s11 * a02);
    const T q3 = J2 * (T(1) / T(3));
    const T ip = frsqrt(q3);
    const T p = q3 * ip;
    T r = T(0.5) * J3 * ip * ip * ip;
    r = r > T(1) ? T(1) : (r < T(-1) ? T(-1) : r);
    T c = seed_cos_third<T>(r);
    const T den = T(12) * c * c - T(3);
    if (den > T(1e-3)) c -= (T(4) * c * c * c - T(3) * c - r) * frcp(den);
    c = c > T(1) ? T(1) : (c < T(0.5) ? T(0.5) : c);
    const T x = T(1) - c * c;
    const T sn = x > T(0) ? x * frsqrt(x) : T(0);
    const T lmax = m + T(2) * p * c;
    const T lmin = m + T(2) * p * (T(-0.5) * c - T(0.86602540378443864676) * sn);
    const T lmid = T(3) * m - lmax - lmin;
    const T iso = (lmax - lmid >= lmid - lmin) ? lmax : lmin;
    // null vector of A - iso I: largest cross product of two rows
    const T r0[3] = {a00 - iso, a01, a02}, r1[3] = {a01, a11 - iso, a12}, r2[3] = {a02, a12, a22 - iso};
    T v[3], w[3];
    v[0] = r0[1] * r1[2] - r0[2] * r1[1];
    v[1] = r0[2] * r1[0] - r0[0] * r1[2];
    v[2] = r0[0] * r1[1] - r0[1] * r1[0];
    T nv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    w[0] = r0[1] * r2[2] - r0[2] * r2[1];
    w[1] = r0[2] * r2[0] - r0[0] * r2[2];
    w[2] = r0[0] * r2[1] - r0[1] * r2[0];
    T nw = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    if (nw > nv) { v[0] = w[0]; v[1] = w[1]; v[2] = w[2]; nv = nw; }
    w[0] = r1[1] * r2[2] - r1[2] * r2[1];
    w[1] = r1[2] * r2[0] - r1[0] * r2[2];
    w[2] = r1[0] * r2[1] - r1[1] * r2[0];
    nw = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    if (nw > nv) { v[0] = w[0]; v[1] = w[1]; v[2] = w[2]; nv = nw; }
    if (nv > Eps<T>::tiny) {
      const T in = frsqrt(nv);
      const T n3[3] = {v[0] * in, v[1] * in, v[2] * in};
      // completion: n3 x e_k for the axis k where |n3_k| is smallest
      const T ax = pf_abs(n3[0]), ay = pf_abs(n3[1]), az = pf_abs(n3[2]);
      T u1[3];
      if (ax <= ay && ax <= az) { u1[0] = T(0); u1[1] = n3[2]; u1[2] = -n3[1]; }
      else if (ay <= az) { u1[0] = -n3[2]; u1[1] = T(0); u1[2] = n3[0]; }
      else { u1[0] = n3[1]; u1[1] = -n3[0]; u1[2] = T(0); }
      const T iu = frsqrt(u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]);
      u1[0] *= iu; u1[1] *= iu; u1[2] *= iu;
      const T u2[3] = {n3[1] * u1[2] - n3[2] * u1[1], n3[2] * u1[0] - n3[0] * u1[2], n3[0] * u1[1] - n3[1] * u1[0]};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        V[3 * k + 0] = u1[k];
        V[3 * k + 1] = u2[k];
        V[3 * k + 2] = n3[k];
      }
    }
  }
  // B = V^T A V
  const T Am[9] = {a00, a01, a02, a01, a11, a12, a02, a12, a22};
  T W[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) W[3 * i + j] = Am[3 * i] * V[j] + Am[3 * i + 1] * V[3 + j] + Am[3 * i + 2] * V[6 + j];
  T b[6];
  const int ri[6] = {0, 1, 2, 1, 0, 0}, ci[6] = {0, 1, 2, 2, 2, 1};
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int i = ri[k], j = ci[k];
    b[k] = V[i] * W[j] + V[3 + i] * W[3 + j] + V[6 + i] * W[6 + j];
  }
  T b00 = b[0], b11 = b[1], b22 = b[2], b12 = b[3], b02 = b[4], b01 = b[5];
  jacobi_rotate(b00, b11, b01, b02, b12, V, 0, 1);
  // The isolated vector's couplings b02, b12 are of the order of the closed form's
  // error. Where they are below 1e-15 of the gaps on every lane of the wave, the two
  // rotations would turn V by less than that angle; they are skipped as a whole.
  const bool small = pf_abs(b02) <= T(1e-15) * pf_abs(b22 - b00) && pf_abs(b12) <= T(1e-15) * pf_abs(b22 - b11);
  if (!__all(small)) {
    jacobi_rotate(b00, b22, b02, b01, b12, V, 0, 2);
    jacobi_rotate(b11, b22, b12, b01, b02, V, 1, 2);
  }
  lam[0] = b00;
  lam[1] = b11;
  lam[2] = b22;
}

// (ln b_i - ln b_j) / (b_i - b_j) for b = 1 + beta, finite at b_i == b_j.
// With x = b_i / b_j - 1 and z = x / (2 + x): ln(b_i/b_j) = 2 atanh(z), so the
// quotient is 2/(2 + x) atanh(z)/z / b_j (series for |x| <= 0.25); beyond that the
// logarithms are far enough apart for the plain difference quotient.
template <typename T>
__device__ inline T log_divdiff(T beta_i, T beta_j, T eps_i, T eps_j, T ib_j) {
  const T x = (beta_i - beta_j) * ib_j;
  T r;
  if (pf_abs(x) <= Eps<T>::series) {
    const T w = frcp(T(2) + x);
    const T zz = x * w;
    r = T(2) * w * atanh_ratio(zz * zz) * ib_j;
  } else {
    r = T(2) * (eps_i - eps_j) * frcp(beta_i - beta_j);
  }
  return r;
}

// Everything the tangent needs at one point (residual pass output).
template <typename T> struct QPState {
  T Fi[9];      // F^-1
  T b[6];       // b_tr = I + A
  T N[9];       // eigenvectors of b_tr (columns)
  T bd[3];      // principal values b_i of b_tr
  T hinv[3];    // 1 / (2 b_i)
  T e[3];       // deviatoric principal trial log strain
  T theta;      // tr eps
  T g, gp;      // degradation and its derivative
  T c;          // radial-return factor
  T kq, kphi;   // plastic tangent: d(c e)_i = c de_i + e_i (kq e.de + kphi dphi)
  T taub[3];    // block principal Kirchhoff stress (undegraded)
  T taud[3];    // degraded principal Kirchhoff stress
  T coef[3];    // off-diagonal tangent factors for pairs (1,2), (0,2), (0,1)
  T tau[6];     // degraded Kirchhoff stress tau_degr
  T psi, H, L;  // psi^+, max(H_n, psi^+), local phase-field residual
  T dLcoef;     // dL / dphi at fixed history
  T ddg_s0, ddg_visc;  // d dgamma / d sigma0, d dgamma / d visc (0 when elastic)
  T dg;         // plastic multiplier increment (0 when elastic)
  bool tension, hactive, plastic, bad;
};

// Kinematics at one point (Box 1 step 1, Appendix A): F^-1, b_tr, principal frame,
// principal log strains. G: grad_X u (row-major), st: D[6] (Voigt).
// Returns beta_i and eps_i for the divided differences.
template <typename T>
__device__ inline void qp_kin(const T* G, const T* st, QPState<T>& s, T* beta, T* eps) {
  // F = I + G and its inverse
  T F[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) F[k] = G[k] + ((k % 4 == 0) ? T(1) : T(0));
  const T c00 = F[4] * F[8] - F[5] * F[7];
  const T c01 = F[5] * F[6] - F[3] * F[8];
  const T c02 = F[3] * F[7] - F[4] * F[6];
  const T det = F[0] * c00 + F[1] * c01 + F[2] * c02;
  const T idet = frcp(det);
  s.Fi[0] = c00 * idet;
  s.Fi[3] = c01 * idet;
  s.Fi[6] = c02 * idet;
  s.Fi[1] = (F[2] * F[7] - F[1] * F[8]) * idet;
  s.Fi[4] = (F[0] * F[8] - F[2] * F[6]) * idet;
  s.Fi[7] = (F[1] * F[6] - F[0] * F[7]) * idet;
  s.Fi[2] = (F[1] * F[5] - F[2] * F[4]) * idet;
  s.Fi[5] = (F[2] * F[3] - F[0] * F[5]) * idet;
  s.Fi[8] = (F[0] * F[4] - F[1] * F[3]) * idet;

  // A = b_tr - I = G + G^T + G G^T + F D F^T  (eq:inelasticity-be-update, Cin^-1 = I + D)
  T A[6];
  const int ri[6] = {0, 1, 2, 1, 0, 0}, ci[6] = {0, 1, 2, 2, 2, 1};
  T FD[9];
  {
    const T D00 = st[0], D11 = st[1], D22 = st[2], D12 = st[3], D02 = st[4], D01 = st[5];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const T f0 = F[3 * i], f1 = F[3 * i + 1], f2 = F[3 * i + 2];
      FD[3 * i + 0] = f0 * D00 + f1 * D01 + f2 * D02;
      FD[3 * i + 1] = f0 * D01 + f1 * D11 + f2 * D12;
      FD[3 * i + 2] = f0 * D02 + f1 * D12 + f2 * D22;
    }
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int i = ri[k], j = ci[k];
    T v = G[3 * i + j] + G[3 * j + i];
#pragma unroll
    for (int l = 0; l < 3; ++l) v += G[3 * i + l] * G[3 * j + l] + FD[3 * i + l] * F[3 * j + l];
    A[k] = v;
    s.b[k] = v + ((k < 3) ? T(1) : T(0));
  }
  // principal values and frame (eq:inelasticity-spectral-decomposition)
  eig_sym3(A, beta, s.N);
  s.bad = !(det > T(0)) || !(beta[0] > T(-1)) || !(beta[1] > T(-1)) || !(beta[2] > T(-1));
  // principal trial log strains with log1p (eq:inelasticity-log-strain-principal)
  s.theta = T(0);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    eps[i] = half_log1p(beta[i]);
    s.bd[i] = T(1) + beta[i];
    s.hinv[i] = T(0.5) * frcp(s.bd[i]);
    s.theta += eps[i];
  }
  const T th3 = s.theta * (T(1) / T(3));
#pragma unroll
  for (int i = 0; i < 3; ++i) s.e[i] = eps[i] - th3;
}

// Degraded Kirchhoff stress in the global frame and the off-diagonal tangent
// factors g mu c (ln b_i - ln b_j)/(b_i - b_j), from the principal quantities.
template <typename T>
__device__ inline void qp_frame_stress(const MatParams<T>& m, const T* beta, const T* eps, QPState<T>& s) {
  const int ri[6] = {0, 1, 2, 1, 0, 0}, ci[6] = {0, 1, 2, 2, 2, 1};
  const T* N = s.N;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int i = ri[k], j = ci[k];
    s.tau[k] = s.taud[0] * N[3 * i] * N[3 * j] + s.taud[1] * N[3 * i + 1] * N[3 * j + 1] +
               s.taud[2] * N[3 * i + 2] * N[3 * j + 2];
  }
  const T gmc = s.g * m.mu * s.c;
  s.coef[0] = gmc * log_divdiff(beta[1], beta[2], eps[1], eps[2], T(2) * s.hinv[2]);
  s.coef[1] = gmc * log_divdiff(beta[0], beta[2], eps[0], eps[2], T(2) * s.hinv[2]);
  s.coef[2] = gmc * log_divdiff(beta[0], beta[1], eps[0], eps[1], T(2) * s.hinv[1]);
}

// Residual state at one point: steps of Box 1 / Box 2 and Section 3.
//   G: grad_X u (row-major), phi: phase field at the point, phin: previous phi,
//   st: D[6] (Voigt), ebar_p, H_n.
//   VOCE = false compiles the linear-hardening return only (kernels launched for
//   contexts without a Voce phase, so that the iteration widens no register budget);
//   MAXW = true adds the Maxwell update of a branch with m.am > 0.
template <typename T, bool VOCE = true, bool MAXW = false>
__device__ inline void qp_state(const MatParams<T>& m, const FracParams<T>& fr, const T* G, T phi,
                                T phin, const T* st, QPState<T>& s) {
  T beta[3], eps[3];
  qp_kin<T>(G, st, s, beta, eps);
  // degradation (eq:degr-funct)
  const T omp = T(1) - phi;
  s.g = omp * omp + fr.eta;
  s.gp = T(-2) * omp;
  // Prandtl branch with the degraded trial stress (Box 2, eq:degraded-yield-condition)
  const T ee = s.e[0] * s.e[0] + s.e[1] * s.e[1] + s.e[2] * s.e[2];
  const T u15 = T(1.5) * ee;
  const T q = (u15 > T(0)) ? T(2) * m.mu * u15 * frsqrt(u15) : T(0);
  const T sn = VOCE ? yield_stress(m, st[6]) : m.sigma0 + m.H * st[6];
  const T f = s.g * q - sn;
  s.plastic = m.plastic && (f > T(0));
  s.c = T(1);
  s.kq = T(0);
  s.kphi = T(0);
  s.ddg_s0 = T(0);
  s.ddg_visc = T(0);
  s.dg = T(0);
  if (s.plastic) {
    const T iq = frcp(q);
    T dg;
    if (VOCE && m.bv > T(0)) {
      // Voce: Box 2's Newton iteration on g q - 3 g mu dg - sigma_y(ebar_n + dg)(1 + a dg) = 0
      // from dg = 0, kept inside [0, q / (3 mu)] (positive, resp. negative, at the ends)
      // by bisection when a step leaves it; bounded, lanes finish independently
      T lo = T(0), hi = q / (T(3) * m.mu), d = T(0);
      for (int it = 0; it < 200; ++it) {
        const T sy = yield_stress(m, st[6] + d), hy = yield_slope(m, st[6] + d);
        const T ft = s.g * q - T(3) * s.g * m.mu * d - sy * (T(1) + m.a * d);
        if (ft > T(0)) lo = d;
        else hi = d;
        T nd = d + ft / (T(3) * s.g * m.mu + hy * (T(1) + m.a * d) + m.a * sy);
        if (!(nd > lo && nd < hi)) nd = T(0.5) * (lo + hi);
        const T step = fabs(nd - d);
        d = nd;
        if (step <= T(1e-15) * d || hi - lo <= T(1e-15) * hi) break;
      }
      dg = d;
    } else {
      // linear hardening: the smaller positive root in closed form (stable)
      const T B = T(3) * s.g * m.mu + m.H + m.a * sn;
      const T disc = B * B + T(4) * m.a * m.H * f;
      dg = T(2) * f * frcp(B + disc * frsqrt(disc));
    }
    s.dg = dg;
    s.c = T(1) - T(3) * m.mu * dg * iq;
    const T ep = st[6] + dg;
    const T sy = VOCE ? yield_stress(m, ep) : sn + m.H * dg;
    const T den = T(3) * s.g * m.mu + (VOCE ? yield_slope(m, ep) : m.H) * (T(1) + m.a * dg) + m.a * sy;
    const T iden = frcp(den);
    const T w = T(3) * m.mu * iq;
    s.kq = -w * (s.g * iden - dg * iq) * (T(6) * m.mu * m.mu * iq);
    s.kphi = -w * s.gp * (q - T(3) * m.mu * dg) * iden;
    s.ddg_s0 = -(T(1) + m.a * dg) * ((VOCE && m.bv > T(0)) ? exp(-m.bv * ep) : T(1)) * iden;
    s.ddg_visc = -sy * dg * fr.inv_dt * iden;
  }
  if (MAXW && m.am > T(0)) {
    // Maxwell branch with the degraded modulus g mu: eps_d^e = c eps_d^e,tr with
    // c = 1 / (1 + g mu dt / eta_d) and dc/dphi = -(mu dt / eta_d) g' c^2
    // (eq:principal-directions-format-1, eq:maxwell-dtau-dphi)
    s.c = frcp(T(1) + m.am * s.g);
    s.kphi = -m.am * s.gp * s.c * s.c;
  }
  // block stress, Amor split, psi^+ (eq:principal-stress-update-eigenvalues,
  // eq:linear-degraded-stress, principal psi^+ of Appendix A)
  s.tension = s.theta >= T(0);
  const T kt = m.kappa * s.theta;
  const T tmu = T(2) * m.mu * s.c;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    s.taub[i] = tmu * s.e[i] + kt;
    s.taud[i] = s.tension ? s.g * s.taub[i] : s.g * (tmu * s.e[i]) + kt;
  }
  s.psi = m.mu * s.c * s.c * ee + (s.tension ? T(0.5) * kt * s.theta : T(0));
  // history (Miehe): strict switch
  s.hactive = s.psi > st[7];
  s.H = s.hactive ? s.psi : st[7];
  // local phase-field residual (eq:L-viscous) and its phi-derivative (eq:linearized-local-damage-residual)
  const T alpha_p = (fr.at == 2) ? T(2) * phi : T(1);
  const T alpha_pp = (fr.at == 2) ? T(2) : T(0);
  s.L = s.gp * s.H + m.Gc * fr.inv_c0l0 * alpha_p + fr.zeta * (phi - phin) * fr.inv_dt;
  s.dLcoef = T(2) * s.H + m.Gc * fr.inv_c0l0 * alpha_pp + fr.zeta * fr.inv_dt;
  qp_frame_stress<T>(m, beta, eps, s);
}

// Linearisation record of one point, taken in FP64 once per linearisation and
// stored in FP32 (19 values + a flag byte): the return-mapping factor and its
// tangent coefficients, the degradation and the local phase-field coefficient,
// the principal frame of b_tr as a unit quaternion, the principal values b_i,
// the principal log strains and the off-diagonal tangent factors. The FP32
// applies recompute only F^-1 from the FP32 displacement mirror.
// Record slots: return factor, tangent scalars, degradation and its derivative, the
// history term's coefficient, the frame of b_tr as the three smallest components of a
// unit quaternion (the largest, made positive, is recovered from the norm; its index is
// in the flags), the principal trial log strains (b_i = exp(2 eps_i) is recomputed) and
// the off-diagonal divided-difference coefficients.
constexpr int REC_N = 15;
enum RecSlot { R_C = 0, R_KQ, R_KPHI, R_G, R_GP, R_DL, R_Q0, R_E0 = R_Q0 + 3, R_O0 = R_E0 + 3 };
// V = float: the FP32 multigrid record; V = double: the stored FP64 linearisation.
template <typename V> struct LinRecordT {
  V v[REC_N];
  uint8_t flags;  // bit0 tension, bit1 history active, bit2 plastic, bits 3-4 dropped quaternion index
};
using LinRecord = LinRecordT<float>;

// Unit quaternion (w, x, y, z) of a rotation matrix R (row-major), by the
// largest-diagonal-element case split of Shepperd's method (no cancellation).
__device__ inline void rot_to_quat(const double* R, double* q) {
  const double tr = R[0] + R[4] + R[8];
  if (tr > 0.0) {
    const double s = 2.0 * sqrt(tr + 1.0);
    q[0] = 0.25 * s; q[1] = (R[7] - R[5]) / s; q[2] = (R[2] - R[6]) / s; q[3] = (R[3] - R[1]) / s;
  } else if (R[0] > R[4] && R[0] > R[8]) {
    const double s = 2.0 * sqrt(1.0 + R[0] - R[4] - R[8]);
    q[0] = (R[7] - R[5]) / s; q[1] = 0.25 * s; q[2] = (R[1] + R[3]) / s; q[3] = (R[2] + R[6]) / s;
  } else if (R[4] > R[8]) {
    const double s = 2.0 * sqrt(1.0 + R[4] - R[0] - R[8]);
    q[0] = (R[2] - R[6]) / s; q[1] = (R[1] + R[3]) / s; q[2] = 0.25 * s; q[3] = (R[5] + R[7]) / s;
  } else {
    const double s = 2.0 * sqrt(1.0 + R[8] - R[0] - R[4]);
    q[0] = (R[3] - R[1]) / s; q[1] = (R[2] + R[6]) / s; q[2] = (R[5] + R[7]) / s; q[3] = 0.25 * s;
  }
  const double n = 1.0 / sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int k = 0; k < 4; ++k) q[k] *= n;
}

template <typename T>
__device__ inline void quat_to_rot(const T* q, T* R) {
  const T w = q[0], x = q[1], y = q[2], z = q[3];
  const T xx = x * x, yy = y * y, zz = z * z, xy = x * y, xz = x * z, yz = y * z, wx = w * x, wy = w * y, wz = w * z;
  R[0] = T(1) - T(2) * (yy + zz); R[1] = T(2) * (xy - wz);          R[2] = T(2) * (xz + wy);
  R[3] = T(2) * (xy + wz);          R[4] = T(1) - T(2) * (xx + zz); R[5] = T(2) * (yz - wx);
  R[6] = T(2) * (xz - wy);          R[7] = T(2) * (yz + wx);          R[8] = T(1) - T(2) * (xx + yy);
}

template <typename V>
__device__ inline void record_from_state(const QPState<double>& s, LinRecordT<V>& r) {
  r.v[R_C] = (V)s.c;
  r.v[R_KQ] = (V)s.kq;
  r.v[R_KPHI] = (V)s.kphi;
  r.v[R_G] = (V)s.g;
  r.v[R_GP] = (V)s.gp;
  r.v[R_DL] = (V)s.dLcoef;
  // a proper rotation: flipping an eigenvector's sign leaves the tangent unchanged
  double R[9];
  for (int k = 0; k < 9; ++k) R[k] = s.N[k];
  const double det = R[0] * (R[4] * R[8] - R[5] * R[7]) - R[1] * (R[3] * R[8] - R[5] * R[6]) +
                     R[2] * (R[3] * R[7] - R[4] * R[6]);
  if (det < 0.0) R[0] = -R[0], R[3] = -R[3], R[6] = -R[6];
  double q[4];
  rot_to_quat(R, q);
  // q and -q are the same rotation: keep the largest component positive and drop it
  int m = 0;
  for (int k = 1; k < 4; ++k)
    if (fabs(q[k]) > fabs(q[m])) m = k;
  const double sg = q[m] < 0.0 ? -1.0 : 1.0;
  for (int k = 0, o = 0; k < 4; ++k)
    if (k != m) r.v[R_Q0 + o++] = (V)(sg * q[k]);
  const double th3 = s.theta * (1.0 / 3.0);
  for (int i = 0; i < 3; ++i) {
    r.v[R_E0 + i] = (V)(s.e[i] + th3);
    r.v[R_O0 + i] = (V)s.coef[i];
  }
  r.flags = (s.tension ? 1 : 0) | (s.hactive ? 2 : 0) | (s.plastic ? 4 : 0) | (m << 3);
}

// New per-point state after a converged step (Section 2): the elastic log strain
// keeps the trial volumetric part and the return-scaled deviator
// (eq:inelasticity-deviatoric-strain-update-2), b^e = exp(2 eps^e) in the frame of
// b_tr and Cin^-1_{n+1} = F^-1 b^e F^-T (eq:inelasticity-deviatoric-strain-update-3);
// the accumulated plastic strain grows by dgamma
// (eq:plasticity-accumulated-plastic-update) and H = max(H_n, psi^+).
// D = Cin^-1 - I is formed without cancellation as
// F^-1 [sum_i expm1(2 eps^e_i) n_i n_i^T - (G + G^T + G G^T)] F^-T,
// using b^e - F F^T = (b^e - I) - (G + G^T + G G^T).
__device__ inline void commit_from_state(const QPState<double>& s, const double* G, const double* st,
                                         double* out) {
  const double th3 = s.theta * (1.0 / 3.0);
  double ex[3];
  for (int i = 0; i < 3; ++i) ex[i] = expm1(2.0 * (s.c * s.e[i] + th3));
  double M[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double v = ex[0] * s.N[3 * i] * s.N[3 * j] + ex[1] * s.N[3 * i + 1] * s.N[3 * j + 1] +
                 ex[2] * s.N[3 * i + 2] * s.N[3 * j + 2];
      v -= G[3 * i + j] + G[3 * j + i] + G[3 * i] * G[3 * j] + G[3 * i + 1] * G[3 * j + 1] + G[3 * i + 2] * G[3 * j + 2];
      M[3 * i + j] = v;
    }
  // W = F^-1 M F^-T
  double T1[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      T1[3 * i + j] = s.Fi[3 * i] * M[j] + s.Fi[3 * i + 1] * M[3 + j] + s.Fi[3 * i + 2] * M[6 + j];
  const int ri[6] = {0, 1, 2, 1, 0, 0}, ci[6] = {0, 1, 2, 2, 2, 1};
  for (int k = 0; k < 6; ++k) {
    const int i = ri[k], j = ci[k];
    out[k] = T1[3 * i] * s.Fi[3 * j] + T1[3 * i + 1] * s.Fi[3 * j + 1] + T1[3 * i + 2] * s.Fi[3 * j + 2];
  }
  out[6] = st[6] + s.dg;
  out[7] = s.H;
}

// State for the linearised FP32 apply: F^-1 from the FP32 displacement mirror,
// everything else (frame, principal values, decisions, coefficients) from the record.
template <typename T>
__device__ inline void qp_state_lin(const MatParams<T>& m, const T* G, const LinRecordT<T>& r, QPState<T>& s) {
  T F[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) F[k] = G[k] + ((k % 4 == 0) ? T(1) : T(0));
  const T c00 = F[4] * F[8] - F[5] * F[7];
  const T c01 = F[5] * F[6] - F[3] * F[8];
  const T c02 = F[3] * F[7] - F[4] * F[6];
  const T idet = frcp(F[0] * c00 + F[1] * c01 + F[2] * c02);
  s.Fi[0] = c00 * idet;
  s.Fi[3] = c01 * idet;
  s.Fi[6] = c02 * idet;
  s.Fi[1] = (F[2] * F[7] - F[1] * F[8]) * idet;
  s.Fi[4] = (F[0] * F[8] - F[2] * F[6]) * idet;
  s.Fi[7] = (F[1] * F[6] - F[0] * F[7]) * idet;
  s.Fi[2] = (F[1] * F[5] - F[2] * F[4]) * idet;
  s.Fi[5] = (F[2] * F[3] - F[0] * F[5]) * idet;
  s.Fi[8] = (F[0] * F[4] - F[1] * F[3]) * idet;
  {
    const int m = (r.flags >> 3) & 3;
    const T a0 = (T)r.v[R_Q0], a1 = (T)r.v[R_Q0 + 1], a2 = (T)r.v[R_Q0 + 2];
    const T rest = T(1) - (a0 * a0 + a1 * a1 + a2 * a2);
    const T qm = sqrt(rest > T(0) ? rest : T(0));  // >= 1/2 by the choice of m
    const T q[4] = {m == 0 ? qm : a0, m == 1 ? qm : (m == 0 ? a0 : a1), m == 2 ? qm : (m <= 1 ? a1 : a2),
                    m == 3 ? qm : a2};
    quat_to_rot<T>(q, s.N);
  }
  s.c = (T)r.v[R_C];
  s.kq = (T)r.v[R_KQ];
  s.kphi = (T)r.v[R_KPHI];
  s.g = (T)r.v[R_G];
  s.gp = (T)r.v[R_GP];
  s.dLcoef = (T)r.v[R_DL];
  s.tension = r.flags & 1;
  s.hactive = (r.flags >> 1) & 1;
  s.plastic = (r.flags >> 2) & 1;
  s.theta = T(0);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const T E = (T)r.v[R_E0 + i];  // principal trial log strain: b_i = exp(2 E)
    s.bd[i] = fexp(T(2) * E);
    s.hinv[i] = T(0.5) * fexp(T(-2) * E);
    s.theta += E;
    s.coef[i] = (T)r.v[R_O0 + i];
  }
  const T th3 = s.theta * (T(1) / T(3));
#pragma unroll
  for (int i = 0; i < 3; ++i) s.e[i] = (T)r.v[R_E0 + i] - th3;
  const T kt = m.kappa * s.theta;
  const T tmu = T(2) * m.mu * s.c;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    s.taub[i] = tmu * s.e[i] + kt;
    s.taud[i] = s.tension ? s.g * s.taub[i] : s.g * (tmu * s.e[i]) + kt;
  }
}

// First Piola stress P = tau_degr F^-T (eq:mechanical-gradient-transformation).
template <typename T>
__device__ inline void piola(const QPState<T>& s, T* P) {
  const T* t = s.tau;
  const T tm[9] = {t[0], t[5], t[4], t[5], t[1], t[3], t[4], t[3], t[2]};
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int J = 0; J < 3; ++J)
      P[3 * i + J] = tm[3 * i] * s.Fi[3 * J] + tm[3 * i + 1] * s.Fi[3 * J + 1] + tm[3 * i + 2] * s.Fi[3 * J + 2];
}

// Directional derivative (Appendices B-C): (dG, dphi) -> (dP, dL).
// Evaluated in the principal frame of b_tr: with dl = dG F^-1 and Lt = N^T dl N,
// the rotated perturbation N^T (dl b + b dl^T) N is Lt diag(b) + diag(b) Lt^T, and
// dP = N (dtau_rot - diag(tau_d) Lt^T) N^T F^-T, where dtau_rot carries the principal
// increments on the diagonal and the divided-difference terms off it, and the second
// term is the geometric part -tau_degr dl^T expressed in the frame.
// The phase-field gradient term is linear and handled by the caller.
// dpsi: this branch's psi^+ increment, evaluated only when `want` (else 0).
template <typename T>
__device__ inline void qp_tangent_psi(const MatParams<T>& m, const QPState<T>& s, const T* dG, T dphi,
                                      T* dP, T& dpsi, bool want = true) {
  const T* N = s.N;
  // FiN = F^-1 N serves both ends: dl N = dG FiN and F^-T at the output
  T FiN[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      FiN[3 * i + j] = s.Fi[3 * i] * N[j] + s.Fi[3 * i + 1] * N[3 + j] + s.Fi[3 * i + 2] * N[6 + j];
  // Lt = N^T (dl N), dl = dG F^-1
  T dN[9], Lt[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      dN[3 * i + j] = dG[3 * i] * FiN[j] + dG[3 * i + 1] * FiN[3 + j] + dG[3 * i + 2] * FiN[6 + j];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Lt[3 * i + j] = N[i] * dN[j] + N[3 + i] * dN[3 + j] + N[6 + i] * dN[6 + j];
  const T* bd = s.bd;
  // principal strain increments from the diagonal (eq:hencky-stress-linearization)
  T deps[3];
  T dth = T(0);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    deps[i] = Lt[4 * i];  // d eps_i = d b_i / (2 b_i) with d b_i = 2 b_i Lt_ii
    dth += deps[i];
  }
  const T dth3 = dth * (T(1) / T(3));
  T de[3], dce[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) de[i] = deps[i] - dth3;
  // linearised radial return (Box A1 generalised)
  const T kk = s.kq * (s.e[0] * de[0] + s.e[1] * de[1] + s.e[2] * de[2]) + s.kphi * dphi;
#pragma unroll
  for (int i = 0; i < 3; ++i) dce[i] = s.c * de[i] + s.e[i] * kk;
  // degraded principal stress increments (eq:linear-degraded-stress-linearization)
  const T kdt = m.kappa * dth;
  const T tm2 = T(2) * m.mu;
  T X[3], td[3];
  const T kt = m.kappa * s.theta, tmc = tm2 * s.c;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    // block (undegraded) deviatoric and degraded principal stresses, from e, c and theta
    const T taubd = tmc * s.e[i];
    td[i] = s.tension ? s.g * (taubd + kt) : s.g * taubd + kt;
    if (s.tension)
      X[i] = s.g * (tm2 * dce[i] + kdt) + s.gp * dphi * (taubd + kt);
    else
      X[i] = s.g * (tm2 * dce[i]) + kdt + s.gp * dphi * taubd;
  }
  // off-diagonal increments: rotated db_ij times the divided-difference factors
  const T o12 = (Lt[5] * bd[2] + bd[1] * Lt[7]) * s.coef[0];
  const T o02 = (Lt[2] * bd[2] + bd[0] * Lt[6]) * s.coef[1];
  const T o01 = (Lt[1] * bd[1] + bd[0] * Lt[3]) * s.coef[2];
  // Z = dtau_rot - diag(tau_d) Lt^T
  const T Z[9] = {X[0] - td[0] * Lt[0], o01 - td[0] * Lt[3], o02 - td[0] * Lt[6],
                  o01 - td[1] * Lt[1], X[1] - td[1] * Lt[4], o12 - td[1] * Lt[7],
                  o02 - td[2] * Lt[2], o12 - td[2] * Lt[5], X[2] - td[2] * Lt[8]};
  // dP = (N Z N^T) F^-T = (N Z) (F^-1 N)^T
  T NZ[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      NZ[3 * i + j] = N[3 * i] * Z[j] + N[3 * i + 1] * Z[3 + j] + N[3 * i + 2] * Z[6 + j];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int J = 0; J < 3; ++J)
      dP[3 * i + J] = NZ[3 * i] * FiN[3 * J] + NZ[3 * i + 1] * FiN[3 * J + 1] + NZ[3 * i + 2] * FiN[3 * J + 2];
  // psi^+ increment of this branch (eq:energy-displacement-linearization)
  dpsi = T(0);
  if (want) {
    dpsi = tm2 * s.c * (s.e[0] * dce[0] + s.e[1] * dce[1] + s.e[2] * dce[2]);
    if (s.tension) dpsi += m.kappa * s.theta * dth;
  }
}

// The tangent of a single block: dP and the local phase-field increment
// dL = dLcoef dphi + g' dH with dH = dpsi^+ when the history switch is on
// (eq:history-field-linearization, eq:linearized-local-damage-residual).
template <typename T>
__device__ inline void qp_tangent(const MatParams<T>& m, const QPState<T>& s, const T* dG, T dphi,
                                  T* dP, T& dL) {
  T dH;
  qp_tangent_psi<T>(m, s, dG, dphi, dP, dH, s.hactive);
  dL = s.dLcoef * dphi + s.gp * dH;
}

// Reverse (transpose) of qp_tangent: cotangents (Pb = dP-bar, Lb = dL-bar) ->
// (Gb = dG-bar, phib = dphi-bar), step by step in the reverse order of the forward
// map, in the principal frame. Also returns the diagonal of the rotated stress
// cotangent Xd_i = [N^T (Pb F^-1) N]_ii used by the parameter partials.
// Core: Hb = the cotangent of psi^+ (zero when the history switch is off); phib
// starts from phib0 and collects the branch's terms.
template <typename T>
__device__ inline void qp_tangent_T_psi(const MatParams<T>& m, const QPState<T>& s, const T* Pb, T Hb, T phib0,
                                        T* Gb, T& phib, T* Xd) {
  const T* N = s.N;
  const T* bd = s.bd;
  const T tm2 = T(2) * m.mu;
  phib = phib0;
  // FiN = F^-1 N (both ends, as in the forward map)
  T FiN[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      FiN[3 * i + j] = s.Fi[3 * i] * N[j] + s.Fi[3 * i + 1] * N[3 + j] + s.Fi[3 * i + 2] * N[6 + j];
  // dP = (N Z) FiN^T  ->  Zb = N^T (Pb FiN)
  T Zt[9], Zb[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      Zt[3 * i + j] = Pb[3 * i] * FiN[j] + Pb[3 * i + 1] * FiN[3 + j] + Pb[3 * i + 2] * FiN[6 + j];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Zb[3 * i + j] = N[i] * Zt[j] + N[3 + i] * Zt[3 + j] + N[6 + i] * Zt[6 + j];
  Xd[0] = Zb[0];
  Xd[1] = Zb[4];
  Xd[2] = Zb[8];
  // Z = Xfull - diag(tau_d) Lt^T: off-diagonal increments and the geometric term
  // (block deviatoric and degraded principal stresses recomputed from e, c and theta)
  const T kapth = m.kappa * s.theta, tmc = tm2 * s.c;
  T taubd[3], td[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    taubd[i] = tmc * s.e[i];
    td[i] = s.tension ? s.g * (taubd[i] + kapth) : s.g * taubd[i] + kapth;
  }
  T Ltb[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) Ltb[3 * a + b] = -td[b] * Zb[3 * b + a];
  const T ob12 = (Zb[5] + Zb[7]) * s.coef[0];
  const T ob02 = (Zb[2] + Zb[6]) * s.coef[1];
  const T ob01 = (Zb[1] + Zb[3]) * s.coef[2];
  Ltb[5] += bd[2] * ob12;
  Ltb[7] += bd[1] * ob12;
  Ltb[2] += bd[2] * ob02;
  Ltb[6] += bd[0] * ob02;
  Ltb[1] += bd[1] * ob01;
  Ltb[3] += bd[0] * ob01;
  // principal stress increments
  T dceb[3];
  T dthb = T(0);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const T xb = Zb[4 * i];
    dceb[i] = s.g * tm2 * xb;
    if (s.tension) {
      dthb += s.g * m.kappa * xb;
      phib += s.gp * (taubd[i] + kapth) * xb;
    } else {
      dthb += m.kappa * xb;
      phib += s.gp * taubd[i] * xb;
    }
  }
  // psi^+: dpsi = 2 mu c e.dce + tension kappa theta dth
  if (Hb != T(0)) {
#pragma unroll
    for (int i = 0; i < 3; ++i) dceb[i] += tm2 * s.c * s.e[i] * Hb;
    if (s.tension) dthb += kapth * Hb;
  }
  // dce_i = c de_i + e_i (kq e.de + kphi dphi)
  const T sdot = s.e[0] * dceb[0] + s.e[1] * dceb[1] + s.e[2] * dceb[2];
  T deb[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) deb[i] = s.c * dceb[i] + s.kq * sdot * s.e[i];
  phib += s.kphi * sdot;
  // de_i = deps_i - dth/3, dth = sum deps, deps_i = Lt_ii
  const T mdeb = (deb[0] + deb[1] + deb[2]) * (T(1) / T(3));
#pragma unroll
  for (int i = 0; i < 3; ++i) Ltb[4 * i] += deb[i] - mdeb + dthb;
  // Lt = N^T dG FiN  ->  Gb = (N Ltb) FiN^T
  T R[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      R[3 * i + j] = N[3 * i] * Ltb[j] + N[3 * i + 1] * Ltb[3 + j] + N[3 * i + 2] * Ltb[6 + j];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int J = 0; J < 3; ++J)
      Gb[3 * i + J] = R[3 * i] * FiN[3 * J] + R[3 * i + 1] * FiN[3 * J + 1] + R[3 * i + 2] * FiN[3 * J + 2];
}

// Transpose of the single block's tangent: dL = dLcoef dphi + g' dH, dH = dpsi^+ when
// the history switch is on.
template <typename T>
__device__ inline void qp_tangent_T(const MatParams<T>& m, const QPState<T>& s, const T* Pb, T Lb, T* Gb,
                                    T& phib, T* Xd) {
  qp_tangent_T_psi<T>(m, s, Pb, s.hactive ? s.gp * Lb : T(0), s.dLcoef * Lb, Gb, phib, Xd);
}

}  // namespace pfmf
