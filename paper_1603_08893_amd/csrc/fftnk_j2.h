// Finite-strain J2 elasto-plasticity per voxel (de Geus et al. 2017, Sec. 5),
// FP64, for the kernels of libfftnk.
//
// F = Fe Fp; Kirchhoff stress tau = C : ln(be) / 2 with the isotropic C of
// Sec. 4 (bulk K, shear mu); von Mises yield tau_eq - (tau_y0 + H eps_p) <= 0;
// implicit exponential-map return mapping (radial return in principal space
// of the trial be = F Cp^-1 F^T); pull-back P = tau F^-T (Sec. 5.4).  History:
// Cp^-1 as [xx yy zz xy yz xz] and eps_p, 7 doubles per voxel.
// The consistent tangent at frozen history (Sec. 5.3) is applied as a
// directional derivative: the derivative of the matrix logarithm by
// Daleckii-Krein divided differences in the eigenbasis of be, the radial-return
// algorithmic modulus, and the derivative of F^-T.
#pragma once

#include "fftnk_device.h"

namespace fftnk {

struct J2Point {
  double Fi[9];    // F^-1
  double Q[9];     // eigenvectors of the trial be, column a = Q[3 i + a]
  double be[3];    // eigenvalues of the trial be
  double tp[3];    // principal Kirchhoff stress
  double np[3];    // principal flow direction (3/2) dev tau_tr / tau_eq_tr
  double epse[3];  // principal elastic log strain after the return
  double q, dgam;
  int plastic;
};

// Symmetric 3x3 eigen-decomposition by cyclic Jacobi rotations.
// a = [a00 a11 a22 a01 a12 a02] (overwritten by the eigenvalues in a[0..2]),
// V = eigenvectors (columns).  The angle of each rotation zeroes a_pq:
// t = sign(th) / (|th| + sqrt(th^2 + 1)), th = (a_qq - a_pp) / (2 a_pq).
__device__ __forceinline__ void jrot(double& app, double& aqq, double& apq, double& arp, double& arq, double* V,
                                     int p, int q) {
  if (apq == 0.0) return;
  const double th = (aqq - app) / (2.0 * apq);
  const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
  const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
  app -= t * apq;
  aqq += t * apq;
  apq = 0.0;
  const double rp = arp, rq = arq;
  arp = c * rp - s * rq;
  arq = s * rp + c * rq;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double vp = V[3 * i + p], vq = V[3 * i + q];
    V[3 * i + p] = c * vp - s * vq;
    V[3 * i + q] = s * vp + c * vq;
  }
}

__device__ __forceinline__ void eig_sym3(double* a, double* V) {
#pragma unroll
  for (int k = 0; k < 9; ++k) V[k] = (k % 4 == 0) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 16; ++sweep) {
    const double off = a[3] * a[3] + a[4] * a[4] + a[5] * a[5];
    const double dg = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
    if (off == 0.0 || off <= 1e-36 * dg) break;
    jrot(a[0], a[1], a[3], a[5], a[4], V, 0, 1);  // plane (0,1), third index 2: a20 = a02, a21 = a12
    jrot(a[0], a[2], a[5], a[3], a[4], V, 0, 2);  // plane (0,2), third index 1: a10 = a01, a12
    jrot(a[1], a[2], a[4], a[3], a[5], V, 1, 2);  // plane (1,2), third index 0: a01, a02
  }
}

// (ln x - ln y) / (x - y), limit 1/x at x = y
__device__ __forceinline__ double log_divdiff(double x, double y) {
  const double z = (x - y) / y;
  if (fabs(z) < 1e-6) return (1.0 - 0.5 * z + z * z / 3.0) / y;
  return log1p(z) / (x - y);
}

__device__ __forceinline__ void inv33(const double* A, double* B, double& det) {
  const double c00 = A[4] * A[8] - A[5] * A[7], c01 = A[5] * A[6] - A[3] * A[8], c02 = A[3] * A[7] - A[4] * A[6];
  det = A[0] * c00 + A[1] * c01 + A[2] * c02;
  const double id = 1.0 / det;
  B[0] = c00 * id;
  B[3] = c01 * id;
  B[6] = c02 * id;
  B[1] = (A[2] * A[7] - A[1] * A[8]) * id;
  B[4] = (A[0] * A[8] - A[2] * A[6]) * id;
  B[7] = (A[1] * A[6] - A[0] * A[7]) * id;
  B[2] = (A[1] * A[5] - A[2] * A[4]) * id;
  B[5] = (A[2] * A[3] - A[0] * A[5]) * id;
  B[8] = (A[0] * A[4] - A[1] * A[3]) * id;
}

// Return mapping; false when F or the trial be is not admissible.
__device__ __forceinline__ bool j2_return(const double* F, const double* h, double K, double mu, double ty0,
                                          double H, J2Point& s) {
  double det;
  inv33(F, s.Fi, det);
  if (!(det > 0.0)) return false;
  // be = F Cp^-1 F^T (symmetric)
  const double C[9] = {h[0], h[3], h[5], h[3], h[1], h[4], h[5], h[4], h[2]};
  double FC[9];
  mat33<double>(F, C, FC);
  double a[6];
  a[0] = FC[0] * F[0] + FC[1] * F[1] + FC[2] * F[2];
  a[1] = FC[3] * F[3] + FC[4] * F[4] + FC[5] * F[5];
  a[2] = FC[6] * F[6] + FC[7] * F[7] + FC[8] * F[8];
  a[3] = FC[0] * F[3] + FC[1] * F[4] + FC[2] * F[5];
  a[4] = FC[3] * F[6] + FC[4] * F[7] + FC[5] * F[8];
  a[5] = FC[0] * F[6] + FC[1] * F[7] + FC[2] * F[8];
  eig_sym3(a, s.Q);
  double e[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    s.be[k] = a[k];
    if (!(a[k] > 0.0)) return false;
    e[k] = 0.5 * log(a[k]);
  }
  const double tr = e[0] + e[1] + e[2];
  double sd[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) sd[k] = 2.0 * mu * (e[k] - tr / 3.0);
  s.q = sqrt(1.5 * (sd[0] * sd[0] + sd[1] * sd[1] + sd[2] * sd[2]));
  const double phi = s.q - (ty0 + H * h[6]);
  // on or beyond the yield surface the plastic branch applies; on the surface
  // itself dgam = 0 and the tangent is the plastic one-sided derivative
  s.plastic = phi > -1e-12 * ty0 && s.q > 0.0;
  s.dgam = (s.plastic && phi > 0.0) ? phi / (3.0 * mu + H) : 0.0;
  if (s.plastic && !(3.0 * mu + H > 0.0)) return false;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    s.np[k] = s.q > 0.0 ? 1.5 * sd[k] / s.q : 0.0;
    s.tp[k] = K * tr + sd[k] - 2.0 * mu * s.dgam * s.np[k];
    s.epse[k] = e[k] - s.dgam * s.np[k];
  }
  return true;
}

// X = Q diag(d) Q^T
__device__ __forceinline__ void from_principal(const double* Q, const double* d, double* X) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      X[3 * i + j] = Q[3 * i] * d[0] * Q[3 * j] + Q[3 * i + 1] * d[1] * Q[3 * j + 1] + Q[3 * i + 2] * d[2] * Q[3 * j + 2];
}

// P and (optionally) the history after the return; false on failure.
__device__ __forceinline__ bool j2_stress(const double* F, const double* h, double K, double mu, double ty0,
                                          double H, double* P, double* hnew) {
  J2Point s;
  if (!j2_return(F, h, K, mu, ty0, H, s)) return false;
  double tau[9];
  from_principal(s.Q, s.tp, tau);
  // P = tau F^-T: P_ij = tau_ik Fi_jk
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      P[3 * i + j] = tau[3 * i] * s.Fi[3 * j] + tau[3 * i + 1] * s.Fi[3 * j + 1] + tau[3 * i + 2] * s.Fi[3 * j + 2];
  if (hnew) {
    const double ex[3] = {exp(2.0 * s.epse[0]), exp(2.0 * s.epse[1]), exp(2.0 * s.epse[2])};
    double be[9], t[9], Cp[9];
    from_principal(s.Q, ex, be);
    mat33<double>(s.Fi, be, t);
    // Cp^-1 = Fi be Fi^T
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        Cp[3 * i + j] = t[3 * i] * s.Fi[3 * j] + t[3 * i + 1] * s.Fi[3 * j + 1] + t[3 * i + 2] * s.Fi[3 * j + 2];
    hnew[0] = Cp[0];
    hnew[1] = Cp[4];
    hnew[2] = Cp[8];
    hnew[3] = 0.5 * (Cp[1] + Cp[3]);
    hnew[4] = 0.5 * (Cp[5] + Cp[7]);
    hnew[5] = 0.5 * (Cp[2] + Cp[6]);
    hnew[6] = h[6] + s.dgam;
  }
  return true;
}

// Tangent action dP = (dP/dF at frozen history)[dF]; NaN on failure.
__device__ __forceinline__ void j2_tangent(const double* F, const double* h, double K, double mu, double ty0,
                                           double H, const double* dF, double* out) {
  J2Point s;
  if (!j2_return(F, h, K, mu, ty0, H, s)) {
#pragma unroll
    for (int c = 0; c < 9; ++c) out[c] = __builtin_nan("");
    return;
  }
  // dbe = M + M^T, M = dF Cp^-1 F^T
  const double C[9] = {h[0], h[3], h[5], h[3], h[1], h[4], h[5], h[4], h[2]};
  double dFC[9], M[9];
  mat33<double>(dF, C, dFC);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) M[3 * i + j] = dFC[3 * i] * F[3 * j] + dFC[3 * i + 1] * F[3 * j + 1] + dFC[3 * i + 2] * F[3 * j + 2];
  double db[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) db[3 * i + j] = M[3 * i + j] + M[3 * j + i];
  // eigenbasis: dq = Q^T db Q, d eps_ab = 1/2 f(be_a, be_b) dq_ab
  double t1[9], dq[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int j = 0; j < 3; ++j) t1[3 * a + j] = s.Q[a] * db[j] + s.Q[3 + a] * db[3 + j] + s.Q[6 + a] * db[6 + j];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) dq[3 * a + b] = t1[3 * a] * s.Q[b] + t1[3 * a + 1] * s.Q[3 + b] + t1[3 * a + 2] * s.Q[6 + b];
  double de[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) de[3 * a + b] = 0.5 * log_divdiff(s.be[a], s.be[b]) * dq[3 * a + b];
  const double tr = de[0] + de[4] + de[8];
  const double nds = 2.0 * mu * (s.np[0] * (de[0] - tr / 3.0) + s.np[1] * (de[4] - tr / 3.0) + s.np[2] * (de[8] - tr / 3.0));
  const double c1 = s.plastic ? 1.0 - 3.0 * mu * s.dgam / s.q : 1.0;
  const double c2 = s.plastic ? 2.0 * mu * (1.0 / (3.0 * mu + H) - s.dgam / s.q) : 0.0;
  double dt[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      double v = c1 * 2.0 * mu * de[3 * a + b];
      if (a == b) v += K * tr - c1 * 2.0 * mu * tr / 3.0 - c2 * nds * s.np[a];
      dt[3 * a + b] = v;
    }
  // back to the frame: dtau = Q dt Q^T
  double dtau[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int b = 0; b < 3; ++b) t1[3 * i + b] = s.Q[3 * i] * dt[b] + s.Q[3 * i + 1] * dt[3 + b] + s.Q[3 * i + 2] * dt[6 + b];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) dtau[3 * i + j] = t1[3 * i] * s.Q[3 * j] + t1[3 * i + 1] * s.Q[3 * j + 1] + t1[3 * i + 2] * s.Q[3 * j + 2];
  double tau[9];
  from_principal(s.Q, s.tp, tau);
  // G = tau Fi^T dF^T: G_ij = (tau Fi^T)_ik dF_jk; out = (dtau - G) Fi^T
  double A[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      A[3 * i + j] = tau[3 * i] * s.Fi[3 * j] + tau[3 * i + 1] * s.Fi[3 * j + 1] + tau[3 * i + 2] * s.Fi[3 * j + 2];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      t1[3 * i + j] = dtau[3 * i + j] - (A[3 * i] * dF[3 * j] + A[3 * i + 1] * dF[3 * j + 1] + A[3 * i + 2] * dF[3 * j + 2]);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      out[3 * i + j] = t1[3 * i] * s.Fi[3 * j] + t1[3 * i + 1] * s.Fi[3 * j + 1] + t1[3 * i + 2] * s.Fi[3 * j + 2];
}

// The compact tangent at F (frozen history): everything of the tangent action
// that does not depend on dF, computed once per linearisation point (see
// kJ2Tan).  With f_ab the divided differences of ln in the eigenvalues of the
// trial be, the principal increments are dt_ab = G_ab dq_ab (a != b) and
// dt_aa = sum_b D_ab dq_bb for dq = Q^T dbe Q.  false (and NaN data) where the
// return mapping fails.
__device__ __forceinline__ bool j2_tangent_data(const double* F, const double* h, double K, double mu, double ty0,
                                                double H, double* t) {
  J2Point s;
  if (!j2_return(F, h, K, mu, ty0, H, s)) {
#pragma unroll
    for (int k = 0; k < kJ2Tan; ++k) t[k] = __builtin_nan("");
    return false;
  }
  const double c1 = s.plastic ? 1.0 - 3.0 * mu * s.dgam / s.q : 1.0;
  const double c2 = s.plastic ? 2.0 * mu * (1.0 / (3.0 * mu + H) - s.dgam / s.q) : 0.0;
  const double nsum = s.np[0] + s.np[1] + s.np[2];
#pragma unroll
  for (int k = 0; k < 9; ++k) t[k] = s.Q[k];
  t[9] = c1 * mu * log_divdiff(s.be[0], s.be[1]);
  t[10] = c1 * mu * log_divdiff(s.be[1], s.be[2]);
  t[11] = c1 * mu * log_divdiff(s.be[0], s.be[2]);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const double m = (a == b ? c1 * 2.0 * mu : 0.0) + K - c1 * 2.0 * mu / 3.0 -
                       c2 * 2.0 * mu * s.np[a] * (s.np[b] - nsum / 3.0);
      t[12 + 3 * a + b] = m * 0.5 * log_divdiff(s.be[b], s.be[b]);
    }
#pragma unroll
  for (int k = 0; k < 3; ++k) t[21 + k] = s.tp[k];
  return true;
}

// Tangent action dP = (dP/dF at frozen history)[dF] from the compact tangent t
// at F (same steps as j2_tangent after its return mapping).
__device__ __forceinline__ void j2_tangent_compact(const double* F, const double* h, const double* t, const double* dF,
                                                   double* out) {
  double Fi[9], det;
  inv33(F, Fi, det);
  const double* Q = t;
  const double C[9] = {h[0], h[3], h[5], h[3], h[1], h[4], h[5], h[4], h[2]};
  double dFC[9], M[9];
  mat33<double>(dF, C, dFC);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) M[3 * i + j] = dFC[3 * i] * F[3 * j] + dFC[3 * i + 1] * F[3 * j + 1] + dFC[3 * i + 2] * F[3 * j + 2];
  double db[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) db[3 * i + j] = M[3 * i + j] + M[3 * j + i];
  double t1[9];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int j = 0; j < 3; ++j) t1[3 * a + j] = Q[a] * db[j] + Q[3 + a] * db[3 + j] + Q[6 + a] * db[6 + j];
  auto dq = [&](int a, int b) { return t1[3 * a] * Q[b] + t1[3 * a + 1] * Q[3 + b] + t1[3 * a + 2] * Q[6 + b]; };
  const double q00 = dq(0, 0), q11 = dq(1, 1), q22 = dq(2, 2);
  double dt[9];
  dt[0] = t[12] * q00 + t[13] * q11 + t[14] * q22;
  dt[4] = t[15] * q00 + t[16] * q11 + t[17] * q22;
  dt[8] = t[18] * q00 + t[19] * q11 + t[20] * q22;
  dt[1] = dt[3] = t[9] * dq(0, 1);
  dt[5] = dt[7] = t[10] * dq(1, 2);
  dt[2] = dt[6] = t[11] * dq(0, 2);
  // dtau = Q dt Q^T, tau = Q diag(tp) Q^T
  double dtau[9], tau[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int b = 0; b < 3; ++b) t1[3 * i + b] = Q[3 * i] * dt[b] + Q[3 * i + 1] * dt[3 + b] + Q[3 * i + 2] * dt[6 + b];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) dtau[3 * i + j] = t1[3 * i] * Q[3 * j] + t1[3 * i + 1] * Q[3 * j + 1] + t1[3 * i + 2] * Q[3 * j + 2];
  from_principal(Q, t + 21, tau);
  double A[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) A[3 * i + j] = tau[3 * i] * Fi[3 * j] + tau[3 * i + 1] * Fi[3 * j + 1] + tau[3 * i + 2] * Fi[3 * j + 2];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      t1[3 * i + j] = dtau[3 * i + j] - (A[3 * i] * dF[3 * j] + A[3 * i + 1] * dF[3 * j + 1] + A[3 * i + 2] * dF[3 * j + 2]);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      out[3 * i + j] = t1[3 * i] * Fi[3 * j] + t1[3 * i + 1] * Fi[3 * j + 1] + t1[3 * i + 2] * Fi[3 * j + 2];
}

}  // namespace fftnk

namespace fftnk {

// J2 parameters and committed history of global voxel gv
__device__ __forceinline__ void j2_point_data(const Material& mat, long long gv, double& K, double& mu, double& ty0,
                                              double& H, double* h) {
  const double* row = mat.table + 4 * mat.phase[gv];
  K = row[0];
  mu = mat.mu_field ? mat.mu_field[gv] : row[1];
  ty0 = row[2];
  H = row[3];
#pragma unroll
  for (int k = 0; k < 7; ++k) h[k] = mat.hist[k * mat.ntot + gv];
}

}  // namespace fftnk
