// fftnk oracle -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, single-threaded FP64 implementation of what the finite-strain
// FFT Newton-Krylov homogenisation method of de Geus, Vondrejc, Zeman, Peerlings
// and Geers ("Finite strain FFT-based non-linear solvers made simple", CMAME 318,
// 2017) computes.  It is the parity reference for the HIP library and shares no
// code, header, table or helper with it.  Only the test suite, the smoke check
// and the benchmark's CPU-baseline leg may load it.
//
// Every routine names the passage of the paper it follows.  Conventions:
//   * a second-order tensor field is stored component-major, [9][n0][n1][n2],
//     component c = 3*i + j holds A_ij, grid axis a2 is the fastest;
//   * grid axis d is the reference direction X_{d+1};
//   * F_ij = dx_i / dX_j (nomenclature appendix).
//
// Parity pins (tests/test_oracle_*.py) check every routine against something
// other than itself: naive DFTs, numpy's FFT, projector invariants, a
// brute-force orthogonal projector built from spectral gradients, closed-form
// hyperelastic states, central finite differences, the paper's fourth-order
// tangent written in its own notation, a 1-D laminate solved by a 3-unknown
// Newton iteration, linear-elastic laminate bounds, and the iteration count the
// paper reports for its cubic-inclusion example.

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>

typedef std::complex<double> cplx;

extern "C" {

// ---------------------------------------------------------------------------
// Status codes and statistics of one increment.
// ---------------------------------------------------------------------------
enum {
  ORC_OK = 0,
  ORC_ECG_MAXIT = 1,
  ORC_ECG_BREAKDOWN = 2,
  ORC_ENEWTON_MAXIT = 3,
  ORC_ENONFINITE = 4,
  ORC_EINVAL = 5,
  ORC_EMATERIAL = 6,
};

#define ORC_MAX_SOLVES 64

typedef struct {
  int status;
  int n_solves;                       // linear solves in the increment (BC solve included)
  int cg_iters[ORC_MAX_SOLVES];       // CG iterations (operator applications) per solve
  double newton_res[ORC_MAX_SOLVES];  // ||dF|| / Fn after each solve
  double cg_relres[ORC_MAX_SOLVES];   // final recursive ||r|| / ||b|| per solve
} orc_stats;

// ---------------------------------------------------------------------------
// 1-D discrete Fourier transforms.
//
// Forward: X[k] = sum_j x[j] exp(-2 pi i j k / n); backward uses +i and is not
// normalised (the 1/n of the inverse is applied by the 3-D driver).
// ---------------------------------------------------------------------------

static int smallest_prime_factor(int n) {
  for (int p = 2; p * p <= n; ++p)
    if (n % p == 0) return p;
  return n;
}

// Recursive decimation-in-time Cooley-Tukey for any n.  The sub-sequences
// x[r], x[r+p], x[r+2p], ... (r = 0..p-1, p the smallest prime factor of n)
// are transformed recursively (length m = n/p), then combined:
//   X[k + m q] = sum_r W_n^{r (k + m q)} Y_r[k],   W_n = exp(sign 2 pi i / n).
// A prime length is done by the naive O(n^2) sum.  The table w[e] holds
// W_N^e for the top-level length N; W_n^e = w[e * N / n].
static void fft_rec(const cplx* in, long stride, cplx* out, int n, int sign,
                    const cplx* w, int N) {
  if (n == 1) {
    out[0] = in[0];
    return;
  }
  const int p = smallest_prime_factor(n);
  const int step = N / n;
  if (p == n) {
    for (int k = 0; k < n; ++k) {
      cplx s = 0.0;
      int e = 0;  // e = j * k mod n, advanced incrementally
      for (int j = 0; j < n; ++j) {
        s += in[j * stride] * w[(long)e * step];
        e += k;
        if (e >= n) e -= n;
      }
      out[k] = s;
    }
    return;
  }
  const int m = n / p;
  for (int r = 0; r < p; ++r) fft_rec(in + r * stride, stride * p, out + (long)r * m, m, sign, w, N);
  std::vector<cplx> tmp(n);
  for (int k = 0; k < m; ++k)
    for (int q = 0; q < p; ++q) {
      const int kk = k + m * q;
      cplx s = 0.0;
      int e = 0;  // e = r * kk mod n
      for (int r = 0; r < p; ++r) {
        s += out[(long)r * m + k] * w[(long)e * step];
        e += kk;
        if (e >= n) e -= n;
      }
      tmp[kk] = s;
    }
  for (int k = 0; k < n; ++k) out[k] = tmp[k];
}

static std::vector<cplx> twiddle_table(int n, int sign) {
  std::vector<cplx> w(n);
  const double two_pi = 6.283185307179586476925286766559;
  for (int e = 0; e < n; ++e) {
    const double a = sign * two_pi * (double)e / (double)n;
    w[e] = cplx(std::cos(a), std::sin(a));
  }
  return w;
}

// In-place 1-D transform of n interleaved complex values (re, im, re, im, ...).
void orc_fft1d(double* data, int n, int sign) {
  cplx* x = reinterpret_cast<cplx*>(data);
  std::vector<cplx> w = twiddle_table(n, sign);
  std::vector<cplx> in(x, x + n), out(n);
  fft_rec(in.data(), 1, out.data(), n, sign, w.data(), n);
  for (int k = 0; k < n; ++k) x[k] = out[k];
}

// Naive 1-D DFT, the pin of orc_fft1d.
void orc_dft1d_naive(const double* in_, double* out_, int n, int sign) {
  const cplx* in = reinterpret_cast<const cplx*>(in_);
  cplx* out = reinterpret_cast<cplx*>(out_);
  const double two_pi = 6.283185307179586476925286766559;
  for (int k = 0; k < n; ++k) {
    cplx s = 0.0;
    for (int j = 0; j < n; ++j) {
      const double a = sign * two_pi * (double)((long)j * k % n) / (double)n;
      s += in[j] * cplx(std::cos(a), std::sin(a));
    }
    out[k] = s;
  }
}

// ---------------------------------------------------------------------------
// 3-D transforms: one 1-D transform per grid line along each axis in turn
// (the separable form the paper notes: 3 x 3 x 3 one-dimensional transforms per
// second-order tensor, Implementation aspects, Sec. 3.3).
// ---------------------------------------------------------------------------

static void fft3d_inplace(cplx* x, int n0, int n1, int n2, int sign) {
  const int dims[3] = {n0, n1, n2};
  const long strides[3] = {(long)n1 * n2, (long)n2, 1};
  for (int ax = 0; ax < 3; ++ax) {
    const int n = dims[ax];
    if (n == 1) continue;
    std::vector<cplx> w = twiddle_table(n, sign);
    std::vector<cplx> line(n), res(n);
    const long s = strides[ax];
    // iterate over all lines along this axis
    const int oa = (ax == 0) ? 1 : 0, ob = (ax == 2) ? 1 : 2;
    for (int ia = 0; ia < dims[oa]; ++ia)
      for (int ib = 0; ib < dims[ob]; ++ib) {
        const long base = (long)ia * strides[oa] + (long)ib * strides[ob];
        for (int t = 0; t < n; ++t) line[t] = x[base + t * s];
        fft_rec(line.data(), 1, res.data(), n, sign, w.data(), n);
        for (int t = 0; t < n; ++t) x[base + t * s] = res[t];
      }
  }
}

void orc_fft3d(double* data, int n0, int n1, int n2, int sign) {
  fft3d_inplace(reinterpret_cast<cplx*>(data), n0, n1, n2, sign);
}

// Naive O(n^2) 3-D DFT: the definition, used to pin orc_fft3d on tiny grids.
void orc_dft3d_naive(const double* in_, double* out_, int n0, int n1, int n2, int sign) {
  const cplx* in = reinterpret_cast<const cplx*>(in_);
  cplx* out = reinterpret_cast<cplx*>(out_);
  const double two_pi = 6.283185307179586476925286766559;
  for (int k0 = 0; k0 < n0; ++k0)
    for (int k1 = 0; k1 < n1; ++k1)
      for (int k2 = 0; k2 < n2; ++k2) {
        cplx s = 0.0;
        for (int j0 = 0; j0 < n0; ++j0)
          for (int j1 = 0; j1 < n1; ++j1)
            for (int j2 = 0; j2 < n2; ++j2) {
              const double ph = (double)((long)j0 * k0 % n0) / n0 + (double)((long)j1 * k1 % n1) / n1 +
                                (double)((long)j2 * k2 % n2) / n2;
              const double a = sign * two_pi * ph;
              s += in[((long)j0 * n1 + j1) * n2 + j2] * cplx(std::cos(a), std::sin(a));
            }
        out[((long)k0 * n1 + k1) * n2 + k2] = s;
      }
}

// ---------------------------------------------------------------------------
// Compatibility projection (Sec. 2.5, equation for G-hat; even grids: App. C;
// properties: App. D).
//
//   G(A) = Re F^{-1}[ G-hat : F(A) ],  (G-hat : A-hat)_ij = xi_j (sum_l xi_l A-hat_il) / |xi|^2
//
// using the double contraction A:B = A_ijkl B_lk of the nomenclature and
// G-hat_ijlm = delta_im xi_j xi_l / |xi|^2.  xi_d = k_d / N_d with k_d the signed
// integer frequency of axis d (for cubic grids the common factor 1/N cancels).
// G-hat is zero at k = 0 (zero-mean property).  A frequency at which some even
// axis sits at its Nyquist index N_d/2 gets one of the two choices of App. C:
// nyq_identity = 0, G-hat = 0 there (the choice that leaves F compatible, the
// paper's default), or nyq_identity = 1, G-hat = identity there (the choice
// that leaves the stress equilibrated).
// Full complex transforms are used (no real-to-complex shortcut).
// ---------------------------------------------------------------------------

static int signed_freq(int idx, int n) { return (2 * idx > n) ? idx - n : idx; }

void orc_project_nyq(int n0, int n1, int n2, const double* A, double* GA, int nyq_identity) {
  const long n = (long)n0 * n1 * n2;
  std::vector<cplx> Ah(9 * n);
  for (int c = 0; c < 9; ++c) {
    for (long v = 0; v < n; ++v) Ah[c * n + v] = cplx(A[c * n + v], 0.0);
    fft3d_inplace(&Ah[c * n], n0, n1, n2, -1);
  }
  for (int i0 = 0; i0 < n0; ++i0)
    for (int i1 = 0; i1 < n1; ++i1)
      for (int i2 = 0; i2 < n2; ++i2) {
        const long v = ((long)i0 * n1 + i1) * n2 + i2;
        const bool nyq = (n0 % 2 == 0 && 2 * i0 == n0) || (n1 % 2 == 0 && 2 * i1 == n1) ||
                         (n2 % 2 == 0 && 2 * i2 == n2);
        const double xi[3] = {(double)signed_freq(i0, n0) / n0, (double)signed_freq(i1, n1) / n1,
                              (double)signed_freq(i2, n2) / n2};
        const double xx = xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2];
        cplx out[9];
        if (xx == 0.0) {
          for (int c = 0; c < 9; ++c) out[c] = 0.0;
        } else if (nyq) {
          for (int c = 0; c < 9; ++c) out[c] = nyq_identity ? Ah[c * n + v] : cplx(0.0);
        } else {
          for (int i = 0; i < 3; ++i) {
            // row i of A-hat projected on xi
            cplx s = 0.0;
            for (int l = 0; l < 3; ++l) s += Ah[(3 * i + l) * n + v] * xi[l];
            for (int j = 0; j < 3; ++j) out[3 * i + j] = s * xi[j] / xx;
          }
        }
        for (int c = 0; c < 9; ++c) Ah[c * n + v] = out[c];
      }
  for (int c = 0; c < 9; ++c) {
    fft3d_inplace(&Ah[c * n], n0, n1, n2, +1);
    for (long v = 0; v < n; ++v) GA[c * n + v] = Ah[c * n + v].real() / (double)n;
  }
}

void orc_project(int n0, int n1, int n2, const double* A, double* GA) { orc_project_nyq(n0, n1, n2, A, GA, 0); }

// ---------------------------------------------------------------------------
// St. Venant-Kirchhoff hyperelasticity (Sec. 4.2):
//   E = (F^T F - I)/2,  S = C : E = lambda tr(E) I + 2 mu E,  P = F . S,
// with the isotropic stiffness parameterised by bulk modulus K and shear
// modulus mu, lambda = K - 2 mu / 3 (the deviatoric split of the example).
// ---------------------------------------------------------------------------

static inline void mat_get(const double* X, long n, long v, double a[9]) {
  for (int c = 0; c < 9; ++c) a[c] = X[c * n + v];
}
static inline void mat_put(double* X, long n, long v, const double a[9]) {
  for (int c = 0; c < 9; ++c) X[c * n + v] = a[c];
}

// Second Piola-Kirchhoff stress of one material point.
static void svk_S(const double F[9], double K, double mu, double S[9]) {
  const double lam = K - 2.0 * mu / 3.0;
  double E[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += F[3 * k + i] * F[3 * k + j];  // (F^T F)_ij
      E[3 * i + j] = 0.5 * (s - (i == j ? 1.0 : 0.0));
    }
  const double trE = E[0] + E[4] + E[8];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) S[3 * i + j] = lam * trE * (i == j ? 1.0 : 0.0) + 2.0 * mu * E[3 * i + j];
}

static void matmul(const double A[9], const double B[9], double C[9]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
      C[3 * i + j] = s;
    }
}

void orc_svk_stress(long n, const double* F, const double* K, const double* mu, double* P) {
  for (long v = 0; v < n; ++v) {
    double f[9], S[9], p[9];
    mat_get(F, n, v, f);
    svk_S(f, K[v], mu[v], S);
    matmul(f, S, p);
    mat_put(P, n, v, p);
  }
}

// Consistent tangent applied to a direction (Sec. 4.3): the linearisation
//   dP = dF . S + F . dS,  dS = C : dE,  dE = (dF^T F + F^T dF)/2,
// which is the action of the paper's fourth-order K = S.I + I^RT:(F.C.F^T):I^RT
// on dF (checked against that form and against finite differences by tests).
void orc_svk_tangent(long n, const double* F, const double* K, const double* mu, const double* dF,
                     double* dP) {
  for (long v = 0; v < n; ++v) {
    double f[9], d[9], S[9];
    mat_get(F, n, v, f);
    mat_get(dF, n, v, d);
    svk_S(f, K[v], mu[v], S);
    const double lam = K[v] - 2.0 * mu[v] / 3.0;
    double dE[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) s += d[3 * k + i] * f[3 * k + j] + f[3 * k + i] * d[3 * k + j];
        dE[3 * i + j] = 0.5 * s;
      }
    const double trdE = dE[0] + dE[4] + dE[8];
    double dS[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) dS[3 * i + j] = lam * trdE * (i == j ? 1.0 : 0.0) + 2.0 * mu[v] * dE[3 * i + j];
    double t1[9], t2[9], out[9];
    matmul(d, S, t1);
    matmul(f, dS, t2);
    for (int c = 0; c < 9; ++c) out[c] = t1[c] + t2[c];
    mat_put(dP, n, v, out);
  }
}

// ---------------------------------------------------------------------------
// Linear algebra helpers over whole fields.
// ---------------------------------------------------------------------------

// Compensated (Kahan) sum of a[i] * b[i].
static double dot(const double* a, const double* b, long m) {
  double s = 0.0, c = 0.0;
  for (long i = 0; i < m; ++i) {
    const double y = a[i] * b[i] - c;
    const double t = s + y;
    c = (t - s) - y;
    s = t;
  }
  return s;
}

static bool all_finite(const double* a, long m) {
  for (long i = 0; i < m; ++i)
    if (!std::isfinite(a[i])) return false;
  return true;
}

// ---------------------------------------------------------------------------
// Material description shared by the routines below: model 0 = St. Venant-
// Kirchhoff with per-voxel (K, mu); model 1 = finite-strain J2 plasticity with
// per-voxel (K, mu, tau_y0, H) and the committed history hist [7][n].
// ---------------------------------------------------------------------------
typedef struct {
  int n0, n1, n2;
  const double* K;
  const double* mu;
  int model;
  const double* ty0;
  const double* H;
  const double* hist;
  int nyq;  // Nyquist choice of the projection (see orc_project_nyq)
  // Krylov method of the linear solves: 0 conjugate gradients; 1 Chebyshev,
  // 2 Richardson, both with the spectral bounds [lo, hi] of A on range(G);
  // 3 GMRES restarted every (int)lo iterations
  int krylov;
  double lo, hi;
} orc_problem;

static int law_stress(const orc_problem& pb, const double* F, double* P, double* hist_new);
static void law_tangent(const orc_problem& pb, const double* F, const double* dF, double* dP);

// The projected-tangent operator of the linearised system (eq. iter:system):
// A p = G( K_(i) applied to p ) with the tangent taken at F_lin.
void orc_apply_operator(int n0, int n1, int n2, const double* K, const double* mu, const double* Flin,
                        const double* p, double* Ap) {
  const long n = (long)n0 * n1 * n2;
  std::vector<double> t(9 * n);
  orc_svk_tangent(n, Flin, K, mu, p, t.data());
  orc_project(n0, n1, n2, t.data(), Ap);
}

// ---------------------------------------------------------------------------
// Conjugate gradients on the projected-tangent operator (Sec. 2.6: a projection
// based Krylov solver that stays compatible; Sec. 3: solved to accuracy eta_CG).
// x0 = 0, r = b, p = r; stop when ||r|| <= eta ||b|| (recursive residual).
// Returns the number of operator applications in *iters.
// ---------------------------------------------------------------------------
static int cg_solve(const orc_problem& pb, const double* Flin, const double* b, double* x, double eta,
                    int max_cg, int* iters, double* relres) {
  const long n = (long)pb.n0 * pb.n1 * pb.n2, m = 9 * n;
  std::vector<double> r(b, b + m), p(b, b + m), w(m);
  for (long i = 0; i < m; ++i) x[i] = 0.0;
  const double bb = dot(b, b, m);
  double rr = bb;
  *iters = 0;
  *relres = 1.0;
  const double stop = eta * std::sqrt(bb);
  if (std::sqrt(rr) <= stop) {
    *relres = 0.0;
    return ORC_OK;
  }
  while (true) {
    if (*iters >= max_cg) return ORC_ECG_MAXIT;
    {
      std::vector<double> t(m);
      law_tangent(pb, Flin, p.data(), t.data());
      orc_project_nyq(pb.n0, pb.n1, pb.n2, t.data(), w.data(), pb.nyq);
    }
    ++*iters;
    const double pw = dot(p.data(), w.data(), m);
    if (!(pw > 0.0) || !std::isfinite(pw)) return ORC_ECG_BREAKDOWN;
    const double alpha = rr / pw;
    for (long i = 0; i < m; ++i) {
      x[i] += alpha * p[i];
      r[i] -= alpha * w[i];
    }
    const double rr_new = dot(r.data(), r.data(), m);
    *relres = std::sqrt(rr_new / bb);
    if (!std::isfinite(rr_new)) return ORC_ENONFINITE;
    if (std::sqrt(rr_new) <= stop) return ORC_OK;
    const double beta = rr_new / rr;
    rr = rr_new;
    for (long i = 0; i < m; ++i) p[i] = r[i] + beta * p[i];
  }
}

// ---------------------------------------------------------------------------
// Other Krylov methods on the same operator (the paper names CG as one choice
// of projection-based Krylov solver, Sec. 2.6; these are the classical
// fixed-coefficient alternatives).  Both need bounds 0 < lo <= hi of the
// spectrum of A on range(G) and no inner product but the stopping test.
//
// Chebyshev iteration (Saad, Iterative Methods for Sparse Linear Systems,
// Sec. 12.1): theta = (hi + lo)/2, delta = (hi - lo)/2, sigma = theta/delta;
// x0 = 0, r0 = b, d0 = r0/theta, rho0 = 1/sigma; then
//   x += d,  r -= A d,  rho' = 1/(2 sigma - rho),  d = rho' rho d + (2 rho'/delta) r.
// The residual is r_k = T_k((theta - A)/delta) r0 / T_k(sigma) (T_k: Chebyshev
// polynomial of the first kind).
//
// Richardson iteration with the optimal fixed step omega = 2/(lo + hi):
//   x += omega r,  r -= omega A r,  so r_k = (I - omega A)^k r0.
//
// Stopping test, iteration count and statuses as in cg_solve.
// ---------------------------------------------------------------------------
static void apply_A(const orc_problem& pb, const double* Flin, const double* p, double* Ap) {
  const long m = 9L * pb.n0 * pb.n1 * pb.n2;
  std::vector<double> t(m);
  law_tangent(pb, Flin, p, t.data());
  orc_project_nyq(pb.n0, pb.n1, pb.n2, t.data(), Ap, pb.nyq);
}

static int chebyshev_solve(const orc_problem& pb, const double* Flin, const double* b, double* x, double eta,
                           int max_it, int* iters, double* relres) {
  const long m = 9L * pb.n0 * pb.n1 * pb.n2;
  *iters = 0;
  *relres = 1.0;
  if (!(pb.lo > 0.0) || !(pb.hi > pb.lo)) return ORC_EINVAL;
  const double theta = 0.5 * (pb.hi + pb.lo), delta = 0.5 * (pb.hi - pb.lo), sigma = theta / delta;
  std::vector<double> r(b, b + m), d(m), Ad(m);
  for (long i = 0; i < m; ++i) {
    x[i] = 0.0;
    d[i] = r[i] / theta;
  }
  const double bb = dot(b, b, m), stop = eta * std::sqrt(bb);
  if (std::sqrt(bb) <= stop) {
    *relres = 0.0;
    return ORC_OK;
  }
  double rho = 1.0 / sigma;
  while (true) {
    if (*iters >= max_it) return ORC_ECG_MAXIT;
    apply_A(pb, Flin, d.data(), Ad.data());
    ++*iters;
    for (long i = 0; i < m; ++i) {
      x[i] += d[i];
      r[i] -= Ad[i];
    }
    const double rr = dot(r.data(), r.data(), m);
    *relres = std::sqrt(rr / bb);
    if (!std::isfinite(rr)) return ORC_ENONFINITE;
    if (std::sqrt(rr) <= stop) return ORC_OK;
    const double rho1 = 1.0 / (2.0 * sigma - rho);
    for (long i = 0; i < m; ++i) d[i] = rho1 * rho * d[i] + (2.0 * rho1 / delta) * r[i];
    rho = rho1;
  }
}

static int richardson_solve(const orc_problem& pb, const double* Flin, const double* b, double* x, double eta,
                            int max_it, int* iters, double* relres) {
  const long m = 9L * pb.n0 * pb.n1 * pb.n2;
  *iters = 0;
  *relres = 1.0;
  if (!(pb.lo > 0.0) || !(pb.hi >= pb.lo)) return ORC_EINVAL;
  const double omega = 2.0 / (pb.lo + pb.hi);
  std::vector<double> r(b, b + m), Ar(m);
  for (long i = 0; i < m; ++i) x[i] = 0.0;
  const double bb = dot(b, b, m), stop = eta * std::sqrt(bb);
  if (std::sqrt(bb) <= stop) {
    *relres = 0.0;
    return ORC_OK;
  }
  while (true) {
    if (*iters >= max_it) return ORC_ECG_MAXIT;
    apply_A(pb, Flin, r.data(), Ar.data());
    ++*iters;
    for (long i = 0; i < m; ++i) {
      x[i] += omega * r[i];
      r[i] -= omega * Ar[i];
    }
    const double rr = dot(r.data(), r.data(), m);
    *relres = std::sqrt(rr / bb);
    if (!std::isfinite(rr)) return ORC_ENONFINITE;
    if (std::sqrt(rr) <= stop) return ORC_OK;
  }
}

// GMRES (Saad, Iterative Methods for Sparse Linear Systems, Alg. 6.9 with the
// Givens-rotation update of Sec. 6.5.3), restarted every m iterations: from
// x0, r = b - A x0, beta = ||r||, v1 = r / beta; Arnoldi with modified
// Gram-Schmidt, w = A v_j, h_ij = <w, v_i>, w -= h_ij v_i (i = 1..j),
// h_{j+1,j} = ||w||, v_{j+1} = w / h_{j+1,j}; the rotations keep H upper
// triangular and |g_{j+1}| is the residual norm of the least-squares iterate;
// at the end of a cycle (or at convergence) x = x0 + V y with H y = g.  The
// iteration count is the number of operator applications, the restarts'
// residual evaluations included.  Same stopping test as CG, on |g|.
static int gmres_solve(const orc_problem& pb, const double* Flin, const double* b, double* x, double eta,
                       int max_it, int m, int* iters, double* relres) {
  const long n9 = 9L * pb.n0 * pb.n1 * pb.n2;
  *iters = 0;
  *relres = 1.0;
  if (m < 1) return ORC_EINVAL;
  for (long i = 0; i < n9; ++i) x[i] = 0.0;
  const double bb = dot(b, b, n9), nb = std::sqrt(bb), stop = eta * nb;
  if (nb <= stop || nb == 0.0) {
    *relres = 0.0;
    return ORC_OK;
  }
  std::vector<std::vector<double>> V(m + 1, std::vector<double>(n9));
  std::vector<double> w(n9), H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
  bool first = true;
  while (true) {
    // residual of the current iterate
    if (first) {
      for (long i = 0; i < n9; ++i) V[0][i] = b[i];
      first = false;
    } else {
      if (*iters >= max_it) return ORC_ECG_MAXIT;
      apply_A(pb, Flin, x, w.data());
      ++*iters;
      for (long i = 0; i < n9; ++i) V[0][i] = b[i] - w[i];
    }
    const double beta = std::sqrt(dot(V[0].data(), V[0].data(), n9));
    *relres = beta / nb;
    if (!std::isfinite(beta)) return ORC_ENONFINITE;
    if (beta <= stop) return ORC_OK;
    for (long i = 0; i < n9; ++i) V[0][i] /= beta;
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;  // columns of this cycle
    bool done = false;
    for (int j = 0; j < m; ++j) {
      if (*iters >= max_it) break;
      apply_A(pb, Flin, V[j].data(), w.data());
      ++*iters;
      for (int i = 0; i <= j; ++i) {
        const double h = dot(w.data(), V[i].data(), n9);
        H[(size_t)i * m + j] = h;
        for (long q = 0; q < n9; ++q) w[q] -= h * V[i][q];
      }
      const double hn = std::sqrt(dot(w.data(), w.data(), n9));
      H[(size_t)(j + 1) * m + j] = hn;
      if (!std::isfinite(hn)) return ORC_ENONFINITE;
      if (hn > 0.0)
        for (long q = 0; q < n9; ++q) V[j + 1][q] = w[q] / hn;
      // earlier rotations on column j, then the one that zeroes h_{j+1,j}
      for (int i = 0; i < j; ++i) {
        const double a = H[(size_t)i * m + j], c2 = H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = cs[i] * a + sn[i] * c2;
        H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c2;
      }
      const double a = H[(size_t)j * m + j], c2 = H[(size_t)(j + 1) * m + j];
      const double d = std::hypot(a, c2);
      cs[j] = a / d;
      sn[j] = c2 / d;
      H[(size_t)j * m + j] = d;
      H[(size_t)(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      k = j + 1;
      *relres = std::fabs(g[j + 1]) / nb;
      if (std::fabs(g[j + 1]) <= stop || hn == 0.0) {
        done = true;
        break;
      }
    }
    // x += V y, H y = g (upper triangular k x k)
    for (int i = k - 1; i >= 0; --i) {
      double t = g[i];
      for (int q = i + 1; q < k; ++q) t -= H[(size_t)i * m + q] * y[q];
      y[i] = t / H[(size_t)i * m + i];
    }
    for (int i = 0; i < k; ++i)
      for (long q = 0; q < n9; ++q) x[q] += y[i] * V[i][q];
    if (done) return ORC_OK;
    if (*iters >= max_it) return ORC_ECG_MAXIT;
  }
}

// Solve A dF = b unless b is at the round-off floor ||b|| <= 1e-14 ||Y|| of the
// field Y that G was applied to; then dF = 0 with zero iterations.
static int cg_or_zero(const orc_problem& pb, const double* Flin, const double* b, const double* Y,
                      double* x, double eta, int max_cg, int* iters, double* relres) {
  const long m = 9L * pb.n0 * pb.n1 * pb.n2;
  const double nb = std::sqrt(dot(b, b, m)), ny = std::sqrt(dot(Y, Y, m));
  if (nb <= 1e-14 * ny || nb == 0.0) {
    for (long i = 0; i < m; ++i) x[i] = 0.0;
    *iters = 0;
    *relres = 0.0;
    return ORC_OK;
  }
  if (pb.krylov == 1) return chebyshev_solve(pb, Flin, b, x, eta, max_cg, iters, relres);
  if (pb.krylov == 2) return richardson_solve(pb, Flin, b, x, eta, max_cg, iters, relres);
  if (pb.krylov == 3) return gmres_solve(pb, Flin, b, x, eta, max_cg, (int)pb.lo, iters, relres);
  return cg_solve(pb, Flin, b, x, eta, max_cg, iters, relres);
}

// ---------------------------------------------------------------------------
// One load increment of Algorithm 1 with a prescribed macroscopic deformation
// gradient (Sec. 3.1 boundary conditions, Sec. 3.2 program structure).
//
//   dFbar = Fbar - mean(F_t)
//   i = 0:  solve G:K(F_t):dF = -G:K(F_t):dFbar (tangent about the start state),
//           F = F_t + dFbar + dF
//   i > 0:  solve G:K(F_i):dF = -G:P(F_i),  F = F_i + dF
//   stop when ||dF|| / ||F_t + dFbar|| < eta_NW and i > 0.
//
// F holds F_t on entry and the converged field on exit (unchanged on failure).
// P receives the stress of the converged field and Pbar its voxel mean.
// ---------------------------------------------------------------------------
static int solve_increment_impl(const orc_problem& pb, double* F, const double* Fbar, double eta_nw,
                                double eta_cg, int max_newton, int max_cg, double* P, double* Pbar,
                                double* hist_new, orc_stats* st) {
  const int n0 = pb.n0, n1 = pb.n1, n2 = pb.n2;
  const long n = (long)n0 * n1 * n2, m = 9 * n;
  orc_stats local;
  if (!st) st = &local;
  std::memset(st, 0, sizeof(*st));
  if (n0 < 1 || n1 < 1 || n2 < 1 || max_newton < 1 || max_newton > ORC_MAX_SOLVES) {
    st->status = ORC_EINVAL;
    return ORC_EINVAL;
  }
  if (!all_finite(Fbar, 9)) {
    st->status = ORC_ENONFINITE;
    return ORC_ENONFINITE;
  }
  std::vector<double> Ft(F, F + m), Fc(F, F + m), Flin(F, F + m), b(m), Y(m), dF(m), Pc(m);
  std::vector<double> hn(pb.model == 1 ? 7 * n : 0);

  // macroscopic increment relative to the mean of the start state
  double dFbar[9];
  for (int c = 0; c < 9; ++c) {
    double s = 0.0, comp = 0.0;
    for (long v = 0; v < n; ++v) {
      const double y = Ft[c * n + v] - comp;
      const double t = s + y;
      comp = (t - s) - y;
      s = t;
    }
    dFbar[c] = Fbar[c] - s / (double)n;
  }
  // BC right-hand side: Y = K(F_t) : dFbar (uniform dFbar field), b = -G(Y)
  {
    std::vector<double> U(m);
    for (int c = 0; c < 9; ++c)
      for (long v = 0; v < n; ++v) U[c * n + v] = dFbar[c];
    law_tangent(pb, Ft.data(), U.data(), Y.data());
    orc_project_nyq(n0, n1, n2, Y.data(), b.data(), pb.nyq);
    for (long i = 0; i < m; ++i) b[i] = -b[i];
  }
  for (int c = 0; c < 9; ++c)
    for (long v = 0; v < n; ++v) Fc[c * n + v] += dFbar[c];
  const double Fn = std::sqrt(dot(Fc.data(), Fc.data(), m));

  int status = ORC_OK;
  for (int it = 0;; ++it) {
    if (it >= max_newton) {
      status = ORC_ENEWTON_MAXIT;
      break;
    }
    int cgit = 0;
    double relres = 0.0;
    status = cg_or_zero(pb, Flin.data(), b.data(), Y.data(), dF.data(), eta_cg, max_cg, &cgit, &relres);
    st->cg_iters[it] = cgit;
    st->cg_relres[it] = relres;
    st->n_solves = it + 1;
    if (status != ORC_OK) break;
    for (long i = 0; i < m; ++i) Fc[i] += dF[i];
    if (!all_finite(Fc.data(), m)) {
      status = ORC_ENONFINITE;
      break;
    }
    status = law_stress(pb, Fc.data(), Pc.data(), hn.empty() ? nullptr : hn.data());
    if (status != ORC_OK) break;
    for (long i = 0; i < m; ++i) Y[i] = Pc[i];
    orc_project_nyq(n0, n1, n2, Pc.data(), b.data(), pb.nyq);
    for (long i = 0; i < m; ++i) b[i] = -b[i];
    const double res = std::sqrt(dot(dF.data(), dF.data(), m)) / Fn;
    st->newton_res[it] = res;
    if (res < eta_nw && it > 0) break;
    Flin = Fc;  // next linearisation point
  }
  st->status = status;
  if (status != ORC_OK) return status;
  for (long i = 0; i < m; ++i) {
    F[i] = Fc[i];
    P[i] = Pc[i];
  }
  if (hist_new && !hn.empty())
    for (long i = 0; i < 7 * n; ++i) hist_new[i] = hn[i];  // "store history variables" (Alg. 1)
  for (int c = 0; c < 9; ++c) {
    double s = 0.0, comp = 0.0;
    for (long v = 0; v < n; ++v) {
      const double y = Pc[c * n + v] - comp;
      const double t = s + y;
      comp = (t - s) - y;
      s = t;
    }
    Pbar[c] = s / (double)n;
  }
  return ORC_OK;
}

int orc_solve_increment(int n0, int n1, int n2, const double* K, const double* mu, double* F,
                        const double* Fbar, double eta_nw, double eta_cg, int max_newton, int max_cg,
                        double* P, double* Pbar, orc_stats* st) {
  orc_problem pb{n0, n1, n2, K, mu, 0, nullptr, nullptr, nullptr, 0, 0, 0.0, 0.0};
  return solve_increment_impl(pb, F, Fbar, eta_nw, eta_cg, max_newton, max_cg, P, Pbar, nullptr, st);
}

// The same increment with the projection's Nyquist choice nyq_identity (App. C;
// see orc_project_nyq): 1 solves with G-hat = identity at Nyquist frequencies.
int orc_solve_increment_nyq(int n0, int n1, int n2, const double* K, const double* mu, double* F,
                            const double* Fbar, double eta_nw, double eta_cg, int max_newton, int max_cg,
                            double* P, double* Pbar, orc_stats* st, int nyq_identity) {
  orc_problem pb{n0, n1, n2, K, mu, 0, nullptr, nullptr, nullptr, nyq_identity ? 1 : 0, 0, 0.0, 0.0};
  return solve_increment_impl(pb, F, Fbar, eta_nw, eta_cg, max_newton, max_cg, P, Pbar, nullptr, st);
}

// One increment with the J2 law (Sec. 5): hist [7][n] holds the committed
// history on entry and, on success only, the history of the converged state.
int orc_solve_increment_j2(int n0, int n1, int n2, const double* K, const double* mu, const double* ty0,
                           const double* H, double* hist, double* F, const double* Fbar, double eta_nw,
                           double eta_cg, int max_newton, int max_cg, double* P, double* Pbar, orc_stats* st) {
  const long n = (long)n0 * n1 * n2;
  std::vector<double> h0(hist, hist + 7 * n);
  orc_problem pb{n0, n1, n2, K, mu, 1, ty0, H, h0.data(), 0, 0, 0.0, 0.0};
  return solve_increment_impl(pb, F, Fbar, eta_nw, eta_cg, max_newton, max_cg, P, Pbar, hist, st);
}

// ---------------------------------------------------------------------------
// Macroscopic tangent and mixed macroscopic control (not in the paper: Sec. 3.1
// prescribes the whole macroscopic deformation gradient and leaves other cases
// to the literature).  Both are built from the boundary-condition system of
// Sec. 3.1 and the operator of Sec. 2.6, unchanged.
//
// Macroscopic tangent at an equilibrium F: a uniform increment E_m of Fbar
// (unit in component m) spreads as E_m + dF with G:K(F):dF = -G:K(F):E_m, the
// boundary-condition solve; so with w the solution of A w = G(K(F):E_m),
//     dPbar/dFbar[:, m] = mean( K(F) : (E_m - w) ).
//
// Mixed control: components m with mask[m] != 0 prescribe Pbar_m = Ptarget_m,
// the others Fbar_m.  Outer Newton iteration on the masked entries of Fbar:
//   solve the deformation-controlled increment at Fbar (Algorithm 1, started
//   from the previous iterate's equilibrium, the load step's start state at
//   first); R = Pbar_M - Ptarget_M; stop when max |R| <= tol_stress; else
//   Fbar_M -= C_MM^{-1} R with C_MM the masked block of the macroscopic
//   tangent at the current equilibrium, its columns solved to CG tolerance
//   max(eta_cg, 1e-4).
// ---------------------------------------------------------------------------

static void mean9(const double* X, long n, double out[9]) {
  for (int c = 0; c < 9; ++c) {
    double s = 0.0, comp = 0.0;
    for (long v = 0; v < n; ++v) {
      const double y = X[c * n + v] - comp;
      const double t = s + y;
      comp = (t - s) - y;
      s = t;
    }
    out[c] = s / (double)n;
  }
}

// columns m with want[m] != 0 of C[i][m] = dPbar_i / dFbar_m at F; appends
// the CG iteration counts to st (when given).  Returns a status.
static int macro_tangent_impl(const orc_problem& pb, const double* F, const int* want, double C[81],
                              double eta_cg, int max_cg, orc_stats* st) {
  const long n = (long)pb.n0 * pb.n1 * pb.n2, m9 = 9 * n;
  std::vector<double> U(m9), Y(m9), b(m9), w(m9), D(m9);
  for (int m = 0; m < 9; ++m) {
    if (!want[m]) continue;
    for (int c = 0; c < 9; ++c)
      for (long v = 0; v < n; ++v) U[c * n + v] = (c == m) ? 1.0 : 0.0;
    law_tangent(pb, F, U.data(), Y.data());
    orc_project_nyq(pb.n0, pb.n1, pb.n2, Y.data(), b.data(), pb.nyq);
    int it = 0;
    double rel = 0.0;
    const int s = cg_or_zero(pb, F, b.data(), Y.data(), w.data(), eta_cg, max_cg, &it, &rel);
    if (st && st->n_solves < ORC_MAX_SOLVES) {
      st->cg_iters[st->n_solves] = it;
      st->cg_relres[st->n_solves] = rel;
      ++st->n_solves;
    }
    if (s != ORC_OK) return s;
    for (long i = 0; i < m9; ++i) U[i] -= w[i];
    law_tangent(pb, F, U.data(), D.data());
    double col[9];
    mean9(D.data(), n, col);
    for (int i = 0; i < 9; ++i) C[9 * i + m] = col[i];
  }
  return ORC_OK;
}

// Solve C x = r for the k x k system held in the leading block (row-major,
// stride k) by Gaussian elimination with partial pivoting.  Returns false if
// a pivot falls to 1e-12 of the largest entry (singular block: the mask leaves
// a direction of Fbar without stress response, e.g. a rigid rotation at zero
// stress).
static bool small_solve(int k, double* C, double* r) {
  double big = 0.0;
  for (int i = 0; i < k * k; ++i) big = std::fmax(big, std::fabs(C[i]));
  for (int j = 0; j < k; ++j) {
    int piv = j;
    for (int i = j + 1; i < k; ++i)
      if (std::fabs(C[i * k + j]) > std::fabs(C[piv * k + j])) piv = i;
    if (!(std::fabs(C[piv * k + j]) > 1e-12 * big)) return false;
    if (piv != j) {
      for (int c = 0; c < k; ++c) std::swap(C[j * k + c], C[piv * k + c]);
      std::swap(r[j], r[piv]);
    }
    for (int i = j + 1; i < k; ++i) {
      const double f = C[i * k + j] / C[j * k + j];
      for (int c = j; c < k; ++c) C[i * k + c] -= f * C[j * k + c];
      r[i] -= f * r[j];
    }
  }
  for (int j = k - 1; j >= 0; --j) {
    double s = r[j];
    for (int c = j + 1; c < k; ++c) s -= C[j * k + c] * r[c];
    r[j] = s / C[j * k + j];
  }
  return true;
}

static int solve_mixed_impl(const orc_problem& pb, double* F, double* Fbar, const int* mask, const double* Ptarget,
                            double tol_stress, int max_outer, double eta_nw, double eta_cg, int max_newton,
                            int max_cg, double* P, double* Pbar, double* hist_new, orc_stats* st, int* outer) {
  const long n = (long)pb.n0 * pb.n1 * pb.n2, m9 = 9 * n;
  orc_stats local;
  if (!st) st = &local;
  std::memset(st, 0, sizeof(*st));
  if (outer) *outer = 0;
  if (max_outer < 1 || !(tol_stress > 0.0)) {
    st->status = ORC_EINVAL;
    return ORC_EINVAL;
  }
  int idx[9], k = 0;
  for (int m = 0; m < 9; ++m)
    if (mask[m]) idx[k++] = m;
  std::vector<double> Fk(F, F + m9), Pk(m9), hk(pb.model == 1 ? 7 * n : 0);
  double Fb[9], Pb[9];
  for (int c = 0; c < 9; ++c) Fb[c] = Fbar[c];
  for (int it = 0; it < max_outer; ++it) {
    if (outer) *outer = it + 1;
    orc_stats inner;
    const int s = solve_increment_impl(pb, Fk.data(), Fb, eta_nw, eta_cg, max_newton, max_cg, Pk.data(), Pb,
                                       hk.empty() ? nullptr : hk.data(), &inner);
    for (int j = 0; j < inner.n_solves && st->n_solves < ORC_MAX_SOLVES; ++j) {
      st->cg_iters[st->n_solves] = inner.cg_iters[j];
      st->cg_relres[st->n_solves] = inner.cg_relres[j];
      st->newton_res[st->n_solves] = inner.newton_res[j];
      ++st->n_solves;
    }
    if (s != ORC_OK) {
      st->status = s;
      return s;
    }
    double R[9], worst = 0.0;
    for (int j = 0; j < k; ++j) {
      R[j] = Pb[idx[j]] - Ptarget[idx[j]];
      worst = std::fmax(worst, std::fabs(R[j]));
    }
    if (!std::isfinite(worst)) {
      st->status = ORC_ENONFINITE;
      return ORC_ENONFINITE;
    }
    if (worst <= tol_stress) {
      for (long i = 0; i < m9; ++i) {
        F[i] = Fk[i];
        P[i] = Pk[i];
      }
      if (hist_new && !hk.empty())
        for (long i = 0; i < 7 * n; ++i) hist_new[i] = hk[i];
      for (int c = 0; c < 9; ++c) {
        Fbar[c] = Fb[c];
        Pbar[c] = Pb[c];
      }
      st->status = ORC_OK;
      return ORC_OK;
    }
    if (it + 1 == max_outer) break;
    // the masked block only steers the outer step: its columns are solved to
    // max(eta_cg, 1e-4) (the stress test, not the tangent, decides convergence)
    double C[81] = {0.0};
    const int sc = macro_tangent_impl(pb, Fk.data(), mask, C, std::fmax(eta_cg, 1e-4), max_cg, st);
    if (sc != ORC_OK) {
      st->status = sc;
      return sc;
    }
    double Cm[81];
    for (int a = 0; a < k; ++a)
      for (int b = 0; b < k; ++b) Cm[a * k + b] = C[9 * idx[a] + idx[b]];
    if (!small_solve(k, Cm, R)) {
      st->status = ORC_EINVAL;
      return ORC_EINVAL;
    }
    for (int j = 0; j < k; ++j) Fb[idx[j]] -= R[j];
  }
  st->status = ORC_ENEWTON_MAXIT;
  return ORC_ENEWTON_MAXIT;
}

// dPbar/dFbar at the equilibrium F (St. Venant-Kirchhoff), columns with want[m].
int orc_macro_tangent(int n0, int n1, int n2, const double* K, const double* mu, const double* F, const int* want,
                      double eta_cg, int max_cg, double* C) {
  orc_problem pb{n0, n1, n2, K, mu, 0, nullptr, nullptr, nullptr, 0, 0, 0.0, 0.0};
  return macro_tangent_impl(pb, F, want, C, eta_cg, max_cg, nullptr);
}

// One increment under mixed control (St. Venant-Kirchhoff).  F: the start
// state on entry, the equilibrium on success (unchanged on failure); Fbar: the
// prescribed entries and the starting guess of the masked ones on entry, the
// solution on success; *outer: outer iterations taken.
int orc_solve_increment_mixed(int n0, int n1, int n2, const double* K, const double* mu, double* F, double* Fbar,
                              const int* mask, const double* Ptarget, double tol_stress, int max_outer,
                              double eta_nw, double eta_cg, int max_newton, int max_cg, double* P, double* Pbar,
                              orc_stats* st, int* outer) {
  orc_problem pb{n0, n1, n2, K, mu, 0, nullptr, nullptr, nullptr, 0, 0, 0.0, 0.0};
  return solve_mixed_impl(pb, F, Fbar, mask, Ptarget, tol_stress, max_outer, eta_nw, eta_cg, max_newton, max_cg,
                          P, Pbar, nullptr, st, outer);
}

// The same with the J2 law: hist as in orc_solve_increment_j2.
int orc_solve_increment_mixed_j2(int n0, int n1, int n2, const double* K, const double* mu, const double* ty0,
                                 const double* H, double* hist, double* F, double* Fbar, const int* mask,
                                 const double* Ptarget, double tol_stress, int max_outer, double eta_nw,
                                 double eta_cg, int max_newton, int max_cg, double* P, double* Pbar, orc_stats* st,
                                 int* outer) {
  const long n = (long)n0 * n1 * n2;
  std::vector<double> h0(hist, hist + 7 * n);
  orc_problem pb{n0, n1, n2, K, mu, 1, ty0, H, h0.data(), 0, 0, 0.0, 0.0};
  return solve_mixed_impl(pb, F, Fbar, mask, Ptarget, tol_stress, max_outer, eta_nw, eta_cg, max_newton, max_cg,
                          P, Pbar, hist, st, outer);
}

// ---------------------------------------------------------------------------
// Adjoint sensitivity of the homogenised stress (not in the paper; derived from
// the boundary-condition system of Sec. 3.1 and the symmetry of G, Sec. 2.3).
//
// At a converged state, G(P(F, mu)) = 0 with F - Fbar in range(G).  A change
// dmu moves P-bar = mean P by mean(K dF + Q dmu), Q = dP/dmu at fixed F, where
// dF in range(G) solves A dF = -G(Q dmu), A = G K.  For a cotangent g (a 3x3
// tensor, dL/dP-bar) the adjoint field w in range(G) solves
//     A w = G(K : g)        (K : g = tangent action on the uniform field g),
// and then, because A is symmetric on range(G),
//     dL/dmu(x) = (1/n) (g - w(x)) : Q_mu(x),   Q_mu = F . 2 dev(E),
//     dL/dK(x)  = (1/n) (g - w(x)) : Q_K(x),    Q_K  = tr(E) F,
// (S = (K - 2 mu/3) tr(E) I + 2 mu E, so dS/dmu = 2 dev E, dS/dK = tr(E) I).
// F is the converged deformation gradient; K, mu the per-voxel moduli.
// Returns the CG status; *iters the CG iterations.
// ---------------------------------------------------------------------------
int orc_adjoint(int n0, int n1, int n2, const double* K, const double* mu, const double* F, const double* g,
                double eta_cg, int max_cg, double* dLdmu, double* dLdK, int* iters) {
  const long n = (long)n0 * n1 * n2, m = 9 * n;
  orc_problem pb{n0, n1, n2, K, mu, 0, nullptr, nullptr, nullptr, 0, 0, 0.0, 0.0};
  std::vector<double> U(m), Y(m), b(m), w(m);
  for (int c = 0; c < 9; ++c)
    for (long v = 0; v < n; ++v) U[c * n + v] = g[c];
  orc_svk_tangent(n, F, K, mu, U.data(), Y.data());
  orc_project(n0, n1, n2, Y.data(), b.data());
  double relres = 0.0;
  const int st = cg_or_zero(pb, F, b.data(), Y.data(), w.data(), eta_cg, max_cg, iters, &relres);
  if (st != ORC_OK) return st;
  for (long v = 0; v < n; ++v) {
    double f[9];
    mat_get(F, n, v, f);
    double E[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) s += f[3 * k + i] * f[3 * k + j];
        E[3 * i + j] = 0.5 * (s - (i == j ? 1.0 : 0.0));
      }
    const double trE = E[0] + E[4] + E[8];
    double D[9];  // 2 dev(E)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) D[3 * i + j] = 2.0 * (E[3 * i + j] - (i == j ? trE / 3.0 : 0.0));
    double Qmu[9];
    matmul(f, D, Qmu);
    double smu = 0.0, sK = 0.0;
    for (int c = 0; c < 9; ++c) {
      const double a = g[c] - w[c * n + v];
      smu += a * Qmu[c];
      sK += a * trE * f[c];
    }
    dLdmu[v] = smu / (double)n;
    if (dLdK) dLdK[v] = sK / (double)n;
  }
  return ORC_OK;
}

// Exposed for tests: one linear solve with the Krylov method `method` (0 CG, 1
// Chebyshev, 2 Richardson; bounds lo, hi for 1 and 2; 3 GMRES restarted every
// (int)lo iterations) at Flin, x0 = 0.
int orc_krylov(int n0, int n1, int n2, const double* K, const double* mu, const double* Flin, const double* b,
               double* x, double eta, int max_it, int method, double lo, double hi, int* iters, double* relres) {
  orc_problem pb{n0, n1, n2, K, mu, 0, nullptr, nullptr, nullptr, 0, method, lo, hi};
  if (method == 1) return chebyshev_solve(pb, Flin, b, x, eta, max_it, iters, relres);
  if (method == 2) return richardson_solve(pb, Flin, b, x, eta, max_it, iters, relres);
  if (method == 3) return gmres_solve(pb, Flin, b, x, eta, max_it, (int)lo, iters, relres);
  return cg_solve(pb, Flin, b, x, eta, max_it, iters, relres);
}

// One increment (St. Venant-Kirchhoff) with the Nyquist choice nyq_identity and
// linear solves by `method`.
int orc_solve_increment_krylov_nyq(int n0, int n1, int n2, const double* K, const double* mu, double* F,
                                   const double* Fbar, double eta_nw, double eta_cg, int max_newton, int max_cg,
                                   double* P, double* Pbar, orc_stats* st, int method, double lo, double hi,
                                   int nyq_identity) {
  orc_problem pb{n0, n1, n2, K, mu, 0, nullptr, nullptr, nullptr, nyq_identity ? 1 : 0, method, lo, hi};
  return solve_increment_impl(pb, F, Fbar, eta_nw, eta_cg, max_newton, max_cg, P, Pbar, nullptr, st);
}

// One increment (St. Venant-Kirchhoff) whose linear solves use `method`.
int orc_solve_increment_krylov(int n0, int n1, int n2, const double* K, const double* mu, double* F,
                               const double* Fbar, double eta_nw, double eta_cg, int max_newton, int max_cg,
                               double* P, double* Pbar, orc_stats* st, int method, double lo, double hi) {
  orc_problem pb{n0, n1, n2, K, mu, 0, nullptr, nullptr, nullptr, 0, method, lo, hi};
  return solve_increment_impl(pb, F, Fbar, eta_nw, eta_cg, max_newton, max_cg, P, Pbar, nullptr, st);
}

// Exposed for tests: plain CG on the operator at a given linearisation point.
int orc_cg(int n0, int n1, int n2, const double* K, const double* mu, const double* Flin, const double* b,
           double* x, double eta, int max_cg, int* iters, double* relres) {
  orc_problem pb{n0, n1, n2, K, mu, 0, nullptr, nullptr, nullptr, 0, 0, 0.0, 0.0};
  return cg_solve(pb, Flin, b, x, eta, max_cg, iters, relres);
}


// ---------------------------------------------------------------------------
// Finite-strain J2 elasto-plasticity (Sec. 5): multiplicative split
// F = Fe Fp, Kirchhoff stress tau = C : ln(be)/2 (logarithmic elastic strain,
// same isotropic C as Sec. 4), von Mises yield tau_eq - (tau_y0 + H eps_p) <= 0
// with linear hardening (Sec. 5.5), associative flow integrated implicitly by
// the exponential map (the elastic-predictor / plastic-corrector scheme the
// paper takes from Simo 1992), P = tau F^-T (pull-back, Sec. 5.4).
// History: C_p^-1 (symmetric, stored xx yy zz xy yz xz) and eps_p.
// ---------------------------------------------------------------------------

typedef double M3[3][3];

static void m3_mul(const M3 A, const M3 B, M3 C) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += A[i][k] * B[k][j];
      C[i][j] = s;
    }
}
static void m3_T(const M3 A, M3 B) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) B[i][j] = A[j][i];
}
static void m3_from9(const double* a, M3 A) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) A[i][j] = a[3 * i + j];
}
static double m3_det(const M3 A) {
  return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
         A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}
static void m3_inv(const M3 A, M3 B) {
  const double d = m3_det(A);
  B[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) / d;
  B[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) / d;
  B[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) / d;
  B[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) / d;
  B[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) / d;
  B[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) / d;
  B[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) / d;
  B[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) / d;
  B[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) / d;
}

// Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix: A = V diag(w) V^T
// (columns of V are the eigenvectors).  Each step applies the plane rotation
// that zeroes one off-diagonal entry (tan of the angle: the small root of
// t^2 + 2 t theta - 1 = 0, theta = (a_qq - a_pp) / (2 a_pq)); sweeps repeat
// until the off-diagonal part is negligible against the diagonal.
void orc_jacobi_eig3(const double* a9, double* w, double* v9) {
  M3 A, V = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  m3_from9(a9, A);
  for (int sweep = 0; sweep < 64; ++sweep) {
    const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    const double diag = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (off == 0.0 || off <= 1e-36 * diag) break;
    const int pairs[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (auto& pq : pairs) {
      const int p = pq[0], q = pq[1];
      if (A[p][q] == 0.0) continue;
      const double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
      const double t = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
      const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
      M3 R = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}}, RT, tmp;
      R[p][p] = c;
      R[q][q] = c;
      R[p][q] = s;
      R[q][p] = -s;
      m3_T(R, RT);
      m3_mul(RT, A, tmp);
      m3_mul(tmp, R, A);
      A[p][q] = A[q][p] = 0.0;
      m3_mul(V, R, tmp);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) V[i][j] = tmp[i][j];
    }
  }
  for (int i = 0; i < 3; ++i) w[i] = A[i][i];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) v9[3 * i + j] = V[i][j];
}

// The divided difference of ln: (ln x - ln y) / (x - y), 1/x at x = y.
static double log_dd(double x, double y) {
  const double z = (x - y) / y;
  if (std::fabs(z) < 1e-6) return (1.0 - z / 2.0 + z * z / 3.0) / y;
  return std::log1p(z) / (x - y);
}

// The return mapping at one point, everything the tangent needs.
typedef struct {
  M3 F, Fi, Q;       // F, F^-1, eigenvectors of the trial be
  double beta[3];    // eigenvalues of the trial be
  double tau_p[3];   // principal Kirchhoff stress
  double n_p[3];     // flow direction N = (3/2) dev tau_tr / tau_eq_tr (principal)
  double q_tr, dgam; // trial equivalent stress, plastic multiplier
  double eps_e[3];   // principal elastic log strain after the return
  int plastic;
} j2_state;

static int j2_return_map(const double* F9, const double* h, double K, double mu, double ty0, double Hh,
                         j2_state* s) {
  m3_from9(F9, s->F);
  const double J = m3_det(s->F);
  if (!(J > 0.0)) return ORC_EMATERIAL;
  m3_inv(s->F, s->Fi);
  const M3 Cpi = {{h[0], h[3], h[5]}, {h[3], h[1], h[4]}, {h[5], h[4], h[2]}};
  M3 FT, t1, be;
  m3_T(s->F, FT);
  m3_mul(s->F, Cpi, t1);
  m3_mul(t1, FT, be);  // trial be = F Cp^-1 F^T
  double be9[9], Q9[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) be9[3 * i + j] = 0.5 * (be[i][j] + be[j][i]);
  orc_jacobi_eig3(be9, s->beta, Q9);
  m3_from9(Q9, s->Q);
  double eps[3];
  for (int a = 0; a < 3; ++a) {
    if (!(s->beta[a] > 0.0)) return ORC_EMATERIAL;
    eps[a] = 0.5 * std::log(s->beta[a]);
  }
  const double tr = eps[0] + eps[1] + eps[2];
  double sdev[3], q2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    sdev[a] = 2.0 * mu * (eps[a] - tr / 3.0);
    q2 += sdev[a] * sdev[a];
  }
  s->q_tr = std::sqrt(1.5 * q2);
  const double phi = s->q_tr - (ty0 + Hh * h[6]);
  // on or beyond the yield surface: plastic branch (at the surface itself,
  // dgam = 0 and the tangent is the plastic one-sided derivative)
  s->plastic = phi > -1e-12 * ty0 && s->q_tr > 0.0;
  s->dgam = 0.0;
  for (int a = 0; a < 3; ++a) s->n_p[a] = s->q_tr > 0.0 ? 1.5 * sdev[a] / s->q_tr : 0.0;
  if (s->plastic) {
    if (!(3.0 * mu + Hh > 0.0)) return ORC_EMATERIAL;
    s->dgam = phi > 0.0 ? phi / (3.0 * mu + Hh) : 0.0;
  }
  for (int a = 0; a < 3; ++a) {
    s->tau_p[a] = K * tr + sdev[a] - 2.0 * mu * s->dgam * s->n_p[a];
    s->eps_e[a] = eps[a] - s->dgam * s->n_p[a];
  }
  return ORC_OK;
}

// P = tau F^-T and (optionally) the updated history of one point.
static int j2_point_stress(const double* F9, const double* h, double K, double mu, double ty0, double Hh,
                           double* P9, double* hnew) {
  j2_state s;
  const int st = j2_return_map(F9, h, K, mu, ty0, Hh, &s);
  if (st != ORC_OK) return st;
  M3 tau = {}, FiT, P;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int a = 0; a < 3; ++a) tau[i][j] += s.Q[i][a] * s.tau_p[a] * s.Q[j][a];
  m3_T(s.Fi, FiT);
  m3_mul(tau, FiT, P);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) P9[3 * i + j] = P[i][j];
  if (hnew) {
    // be = exp(2 eps_e) (coaxial with the trial be), Cp^-1 = F^-1 be F^-T
    M3 be = {}, t1, Cpi;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        for (int a = 0; a < 3; ++a) be[i][j] += s.Q[i][a] * std::exp(2.0 * s.eps_e[a]) * s.Q[j][a];
    m3_mul(s.Fi, be, t1);
    m3_mul(t1, FiT, Cpi);
    hnew[0] = Cpi[0][0];
    hnew[1] = Cpi[1][1];
    hnew[2] = Cpi[2][2];
    hnew[3] = 0.5 * (Cpi[0][1] + Cpi[1][0]);
    hnew[4] = 0.5 * (Cpi[1][2] + Cpi[2][1]);
    hnew[5] = 0.5 * (Cpi[0][2] + Cpi[2][0]);
    hnew[6] = h[6] + s.dgam;
  }
  return ORC_OK;
}

// Consistent tangent at frozen history applied to dF (Sec. 5.3-5.4):
//   dbe = dF Cp^-1 F^T + F Cp^-1 dF^T
//   d eps (eigenbasis of be) = 1/2 f(beta_a, beta_b) (Q^T dbe Q)_ab,  f = divided difference of ln
//   d tau = K tr(d eps) I + 2 mu c1 dev(d eps) - c2 (N : 2 mu dev d eps) N
//           c1 = 1 - 3 mu dgam / q_tr, c2 = 2 mu (1/(3 mu + H) - dgam / q_tr)  (plastic; c1 = 1, c2 = 0 elastic)
//   dP = d tau F^-T - tau F^-T dF^T F^-T
static int j2_point_tangent(const double* F9, const double* h, double K, double mu, double ty0, double Hh,
                            const double* dF9, double* dP9) {
  j2_state s;
  const int st = j2_return_map(F9, h, K, mu, ty0, Hh, &s);
  if (st != ORC_OK) return st;
  const M3 Cpi = {{h[0], h[3], h[5]}, {h[3], h[1], h[4]}, {h[5], h[4], h[2]}};
  M3 dF, dFT, FT, t1, t2, dbe, QT, tmp, dbq;
  m3_from9(dF9, dF);
  m3_T(dF, dFT);
  m3_T(s.F, FT);
  m3_mul(dF, Cpi, t1);
  m3_mul(t1, FT, t2);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) dbe[i][j] = t2[i][j] + t2[j][i];
  m3_T(s.Q, QT);
  m3_mul(QT, dbe, tmp);
  m3_mul(tmp, s.Q, dbq);
  M3 de;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) de[a][b] = 0.5 * log_dd(s.beta[a], s.beta[b]) * dbq[a][b];
  const double tr = de[0][0] + de[1][1] + de[2][2];
  M3 dtp;
  double Nds = 0.0;
  for (int a = 0; a < 3; ++a) Nds += s.n_p[a] * 2.0 * mu * (de[a][a] - tr / 3.0);
  const double c1 = s.plastic ? 1.0 - 3.0 * mu * s.dgam / s.q_tr : 1.0;
  const double c2 = s.plastic ? 2.0 * mu * (1.0 / (3.0 * mu + Hh) - s.dgam / s.q_tr) : 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      const double devd = de[a][b] - (a == b ? tr / 3.0 : 0.0);
      dtp[a][b] = (a == b ? K * tr : 0.0) + c1 * 2.0 * mu * devd - (a == b ? c2 * Nds * s.n_p[a] : 0.0);
    }
  M3 dtau, tau = {}, FiT, out1, out2, t3;
  m3_mul(s.Q, dtp, tmp);
  m3_mul(tmp, QT, dtau);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int a = 0; a < 3; ++a) tau[i][j] += s.Q[i][a] * s.tau_p[a] * s.Q[j][a];
  m3_T(s.Fi, FiT);
  m3_mul(dtau, FiT, out1);
  m3_mul(tau, FiT, t1);
  m3_mul(t1, dFT, t2);
  m3_mul(t2, FiT, t3);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      out2[i][j] = out1[i][j] - t3[i][j];
      dP9[3 * i + j] = out2[i][j];
    }
  return ORC_OK;
}

static void hist_at(const double* hist, long n, long v, double h[7]) {
  for (int k = 0; k < 7; ++k) h[k] = hist[k * n + v];
}

// field versions (exported for the tests)
int orc_j2_stress(long n, const double* F, const double* K, const double* mu, const double* ty0, const double* H,
                  const double* hist, double* P, double* hist_new) {
  for (long v = 0; v < n; ++v) {
    double f[9], h[7], p[9], hn[7];
    mat_get(F, n, v, f);
    hist_at(hist, n, v, h);
    const int st = j2_point_stress(f, h, K[v], mu[v], ty0[v], H[v], p, hist_new ? hn : nullptr);
    if (st != ORC_OK) return st;
    mat_put(P, n, v, p);
    if (hist_new)
      for (int k = 0; k < 7; ++k) hist_new[k * n + v] = hn[k];
  }
  return ORC_OK;
}

int orc_j2_tangent(long n, const double* F, const double* K, const double* mu, const double* ty0, const double* H,
                   const double* hist, const double* dF, double* dP) {
  for (long v = 0; v < n; ++v) {
    double f[9], h[7], d[9], o[9];
    mat_get(F, n, v, f);
    hist_at(hist, n, v, h);
    mat_get(dF, n, v, d);
    const int st = j2_point_tangent(f, h, K[v], mu[v], ty0[v], H[v], d, o);
    if (st != ORC_OK) return st;
    mat_put(dP, n, v, o);
  }
  return ORC_OK;
}

static int law_stress(const orc_problem& pb, const double* F, double* P, double* hist_new) {
  const long n = (long)pb.n0 * pb.n1 * pb.n2;
  if (pb.model == 0) {
    orc_svk_stress(n, F, pb.K, pb.mu, P);
    return ORC_OK;
  }
  return orc_j2_stress(n, F, pb.K, pb.mu, pb.ty0, pb.H, pb.hist, P, hist_new);
}

static void law_tangent(const orc_problem& pb, const double* F, const double* dF, double* dP) {
  const long n = (long)pb.n0 * pb.n1 * pb.n2;
  if (pb.model == 0) {
    orc_svk_tangent(n, F, pb.K, pb.mu, dF, dP);
    return;
  }
  if (orc_j2_tangent(n, F, pb.K, pb.mu, pb.ty0, pb.H, pb.hist, dF, dP) != ORC_OK)
    for (long i = 0; i < 9 * n; ++i) dP[i] = std::nan("");  // a failed point poisons the solve
}
}  // extern "C"
