// CG, Newton and reduction kernels of libfftnk (gfx950).
//
// CG on the projected-tangent operator (de Geus et al. 2017, Sec. 2.6: a
// projection-based Krylov solver that keeps every iterate compatible; Sec. 3:
// solved to accuracy eta_CG), with all scalars resident on the device so that
// iterations can be replayed without host round trips; the Newton-level
// element-wise steps of Algorithm 1 (increment of the macroscopic deformation,
// iterative update F += dF with the constitutive update, homogenised stress);
// and the adjoint gradient.  Every launch covers all RVEs of a context.
// Reductions: block partial sums in fixed slots, summed in a fixed order by one
// work-group per RVE, so results are bitwise reproducible.
#include <utility>

#include "fftnk_device.h"
#include "fftnk_j2.h"

namespace fftnk {


// loop over this work-group's share of the RVE's index range [0, m)
#define FOR_RVE_RANGE(i, m, local, nb) \
  for (long long i = (long long)(local) * kThreads + threadIdx.x; i < (m); i += (long long)(nb) * kThreads)

// The updates x += alpha_j p_j are deferred: the directions of W iterations
// stay in their slots (p_j in slot j mod W, W = Batch::xwin) and the first
// pass of every iteration k with k mod W = 0 applies the W of them, in the
// order of j.  After the last iteration of a solve this kernel applies the
// ones still due, j in [x_lo, x_hi), in the same order.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cg_finish(Batch B, T* __restrict__ x, const T* __restrict__ p,
                                                        const CgState* __restrict__ cg) {
  int local;
  const int rv = find_rve(B, K_ELEM9, blockIdx.x, local);
  const int lo = cptr(cg)[rv].x_lo, hi = cptr(cg)[rv].x_hi, W = B.xwin;
  if (hi <= lo) return;
  const auto& g = grid_of(B, rv);
  const int nb = rve_blocks(B, K_ELEM9, rv);
  const long long m = 9 * g.n, off = 9 * g.vox_off;
  FOR_RVE_RANGE(i, m, local, nb) {
    T v = x[off + i];
    // at most W <= kMaxXWin terms: a fixed unrolled loop keeps their loads in flight together
#pragma unroll
    for (int jj = 0; jj < kMaxXWin; ++jj) {
      const int j = lo + jj;
      if (j < hi) v = v + (T)cptr(cg)[rv].ahist[j % W] * p[(long long)(j % W) * B.vstride + off + i];
    }
    x[off + i] = v;
  }
}


// One work-group per RVE.  A finished RVE (Newton mask) gets done = 1 at once.
// If ||b|| is at the round-off floor of the projected field Y
// (||b|| <= 1e-14 ||Y||, or b = 0) the solve is skipped with dF = 0.
__global__ __launch_bounds__(kThreads) void k_cg_init(Batch B, CgState* cg, double eta, int max_cg, int stall,
                                                      int method, double lo, double hi) {
  const int rv = blockIdx.x;
  CgState& s = cg[rv];
  if (threadIdx.x == 0) {
    // Chebyshev (Saad, Sec. 12.1): theta = (hi + lo)/2, delta = (hi - lo)/2,
    // sigma = theta/delta, rho_0 = 1/sigma, first step gamma_0 = 1/theta
    s.method = method;
    s.lo = lo;
    s.hi = hi;
    s.rho = method == KRYLOV_CHEBYSHEV ? (hi - lo) / (hi + lo) : 0.0;
    s.gam = method == KRYLOV_CHEBYSHEV ? 2.0 / (hi + lo) : 0.0;
  }
  if (B.active && B.active[rv] == 0) {
    if (threadIdx.x == 0) {
      s.done = 1;
      s.iter = 0;
      s.status = ST_OK;
      s.zero_rhs = 1;
      s.x_lo = s.x_hi = 0;
    }
    return;
  }
  const double yy = reduce_range(pslot(B, SLOT_YY), kstart(B, K_ROW1, rv), kstart(B, K_ROW1, rv + 1));
  const double bb = reduce_range(pslot(B, SLOT_BB), kstart(B, K_ROW, rv), kstart(B, K_ROW, rv + 1));
  if (threadIdx.x == 0) {
    s.bb = bb;
    s.rr = bb;
    s.rr_min = bb;
    s.stop2 = eta * eta * bb;
    s.alpha = 0.0;
    s.beta = 0.0;
    s.pw = 0.0;
    s.iter = 0;
    s.since_min = 0;
    s.max_cg = max_cg;
    s.stall_limit = stall;
    s.status = isfinite(bb) ? ST_OK : ST_NONFINITE;
    s.zero_rhs = (bb == 0.0 || sqrt(bb) <= 1e-14 * sqrt(yy)) ? 1 : 0;
    s.x_lo = s.x_hi = 0;
    s.done = (s.zero_rhs || !isfinite(bb) || bb <= s.stop2) ? 1 : 0;
  }
}

__global__ __launch_bounds__(kThreads) void k_cg_beta(Batch B, CgState* cg) {
  const int rv = blockIdx.x;
  CgState& s = cg[rv];
  if (s.done) return;
  const double rr = reduce_range(pslot(B, SLOT_RR), kstart(B, K_ROW, rv), kstart(B, K_ROW, rv + 1));
  if (threadIdx.x == 0) {
    s.iter += 1;
    if (!isfinite(rr)) {
      s.status = ST_NONFINITE;
      s.done = 1;
    } else if (rr <= s.stop2) {
      s.rr = rr;
      s.done = 1;
    } else if (s.iter >= s.max_cg) {
      s.rr = rr;
      s.status = ST_CG_MAXIT;
      s.done = 1;
    } else {
      if (s.method == KRYLOV_CHEBYSHEV) {
        // rho_{k+1} = 1/(2 sigma - rho_k), gamma_{k+1} = 2 rho_{k+1}/delta; with
        // the direction p = d / gamma (d the recurrence's update),
        // beta = rho_{k+1} rho_k gamma_k / gamma_{k+1}
        const double sigma = (s.hi + s.lo) / (s.hi - s.lo), delta = 0.5 * (s.hi - s.lo);
        const double rho1 = 1.0 / (2.0 * sigma - s.rho), gam1 = 2.0 * rho1 / delta;
        s.beta = rho1 * s.rho * s.gam / gam1;
        s.rho = rho1;
        s.gam = gam1;
      } else if (s.method == KRYLOV_RICHARDSON) {
        s.beta = 0.0;
      } else {
        s.beta = rr / s.rr;
      }
      s.rr = rr;
      // progress = the residual norm 13 % below the last recorded minimum
      // (rr below 0.75 of it); at the FP32 rounding floor the residual only
      // fluctuates, and small new minima must not keep the solve alive
      if (rr < 0.75 * s.rr_min) {
        s.rr_min = rr;
        s.since_min = 0;
      } else {
        s.since_min += 1;
      }
      if (s.stall_limit > 0 && s.since_min >= s.stall_limit) s.done = 1;  // stagnation: keep x
    }
  }
}

// ---------------------------------------------------------------------------
// Newton-level element-wise kernels (Alg. 1).
// ---------------------------------------------------------------------------

// Start of an increment: F = F_t (the tangent of the first solve is taken about
// the start state, Sec. 3.1), ||F_t + dFbar||^2 for the convergence test's
// denominator, and the FP32 copy of the linearisation point.
// Ft may be F itself (a solve warm-started from the current iterate).
__global__ __launch_bounds__(kThreads) void k_set_F(Batch B, const double* Ft, double* F, float* __restrict__ Flin32) {
  int local;
  const int rv = find_rve(B, K_VOX, blockIdx.x, local);
  if (skip_rve(B, nullptr, rv)) return;
  const Grid& g = B.grids[rv];
  const int nb = rve_blocks(B, K_VOX, rv);
  const long long n = g.n, off = 9 * g.vox_off;
  const double* u = B.uni + 9 * rv;
  double acc[1] = {0.0};
  FOR_RVE_RANGE(v, n, local, nb) {
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      const double ft = Ft[off + c * n + v];
      F[off + c * n + v] = ft;
      const double f = ft + u[c];
      acc[0] += f * f;
      if (Flin32) Flin32[off + c * n + v] = (float)ft;
    }
  }
  double res[1];
  block_sums<1>(acc, res);
  if (threadIdx.x == 0) pslot(B, SLOT_FF)[blockIdx.x] = res[0];
}

// Stress of the voxel's material law at F; J2 also writes the history of the
// return from the committed state (hnew may be null).  Returns false (and NaN
// stress) where the update is undefined (J2: det F <= 0 or a non-positive
// trial eigenvalue).
template <int LAW>
__device__ __forceinline__ bool stress_at(const Material& mat, long long gv, const double* f, double* Pv, bool hnew) {
  if constexpr (LAW == MODEL_J2) {
    double K, mu, ty0, H, h[7], hn[7];
    j2_point_data(mat, gv, K, mu, ty0, H, h);
    const bool ok = j2_stress(f, h, K, mu, ty0, H, Pv, hn);
    if (!ok) {
#pragma unroll
      for (int c = 0; c < 9; ++c) Pv[c] = __builtin_nan("");
#pragma unroll
      for (int k = 0; k < 7; ++k) hn[k] = h[k];
    }
    if (hnew)
#pragma unroll
      for (int k = 0; k < 7; ++k) mat.hist_new[k * mat.ntot + gv] = hn[k];
    return ok;
  } else {
    double lam, mu, S[9];
    material_at(mat, gv, lam, mu);
    svk_S<double>(f, lam, mu, S);
    mat33<double>(f, S, Pv);
    return true;
  }
}

// F += dF (+ dFbar on the first iteration), constitutive update P = P(F),
// ||dF||^2, the sums of P and the count of voxels whose update failed; the
// next linearisation point in FP32.
template <typename T, int LAW>
__global__ __launch_bounds__(kThreads) void k_newton_update(Batch B, Material mat, double* __restrict__ F,
                                                            const T* __restrict__ x, double* __restrict__ P,
                                                            float* __restrict__ Flin32, int add_uni) {
  int local;
  const int rv = find_rve(B, K_VOX, blockIdx.x, local);
  if (skip_rve(B, nullptr, rv)) return;
  const Grid& g = B.grids[rv];
  const int nb = rve_blocks(B, K_VOX, rv);
  const long long n = g.n, off = 9 * g.vox_off;
  double u[9];
#pragma unroll
  for (int c = 0; c < 9; ++c) u[c] = add_uni ? B.uni[9 * rv + c] : 0.0;
  double acc[11];
#pragma unroll
  for (int k = 0; k < 11; ++k) acc[k] = 0.0;
  FOR_RVE_RANGE(v, n, local, nb) {
    double f[9], Pv[9], d[9];
    // all loads before the first store (F is read and written)
#pragma unroll
    for (int c = 0; c < 9; ++c) d[c] = (double)x[off + c * n + v];
#pragma unroll
    for (int c = 0; c < 9; ++c) f[c] = F[off + c * n + v];
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      f[c] = f[c] + u[c] + d[c];
      F[off + c * n + v] = f[c];
      acc[0] += d[c] * d[c];
      if (Flin32) Flin32[off + c * n + v] = (float)f[c];
    }
    if (!stress_at<LAW>(mat, g.vox_off + v, f, Pv, true)) acc[10] += 1.0;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      P[off + c * n + v] = Pv[c];
      acc[1 + c] += Pv[c];
    }
  }
  double res[11];
  block_sums<11>(acc, res);
  if (threadIdx.x == 0) {
    pslot(B, SLOT_DF)[blockIdx.x] = res[0];
    for (int c = 0; c < 9; ++c) pslot(B, SLOT_PBAR + c)[blockIdx.x] = res[1 + c];
    pslot(B, SLOT_FAIL)[blockIdx.x] = res[10];
  }
}

template <int LAW>
__global__ __launch_bounds__(kThreads) void k_constitutive(Batch B, Material mat, const double* __restrict__ F,
                                                           double* __restrict__ P) {
  int local;
  const int rv = find_rve(B, K_VOX, blockIdx.x, local);
  if (skip_rve(B, nullptr, rv)) return;
  const Grid& g = B.grids[rv];
  const int nb = rve_blocks(B, K_VOX, rv);
  const long long n = g.n, off = 9 * g.vox_off;
  double acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = 0.0;
  FOR_RVE_RANGE(v, n, local, nb) {
    double f[9], Pv[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) f[c] = F[off + c * n + v];
    stress_at<LAW>(mat, g.vox_off + v, f, Pv, false);
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      P[off + c * n + v] = Pv[c];
      acc[c] += Pv[c];
    }
  }
  double res[9];
  block_sums<9>(acc, res);
  if (threadIdx.x == 0)
    for (int c = 0; c < 9; ++c) pslot(B, SLOT_PBAR + c)[blockIdx.x] = res[c];
}

__global__ __launch_bounds__(kThreads) void k_field_sum(Batch B, const double* __restrict__ X, int slot0) {
  int local;
  const int rv = find_rve(B, K_VOX, blockIdx.x, local);
  if (skip_rve(B, nullptr, rv)) return;
  const Grid& g = B.grids[rv];
  const int nb = rve_blocks(B, K_VOX, rv);
  const long long n = g.n, off = 9 * g.vox_off;
  double acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = 0.0;
  FOR_RVE_RANGE(v, n, local, nb) {
#pragma unroll
    for (int c = 0; c < 9; ++c) acc[c] += X[off + c * n + v];
  }
  double res[9];
  block_sums<9>(acc, res);
  if (threadIdx.x == 0)
    for (int c = 0; c < 9; ++c) pslot(B, slot0 + c)[blockIdx.x] = res[c];
}

// out[r * NSLOT + slot0 + s]: grid (nrve, nslots)
__global__ __launch_bounds__(kThreads) void k_reduce(Batch B, int kind, int slot0, double* out) {
  const int rv = blockIdx.x, s = blockIdx.y;
  const double v = reduce_range(pslot(B, slot0 + s), kstart(B, kind, rv), kstart(B, kind, rv + 1));
  if (threadIdx.x == 0) out[rv * NSLOT + slot0 + s] = v;
}

template <typename TI, typename TO>
__global__ __launch_bounds__(kThreads) void k_convert(const TI* __restrict__ in, TO* __restrict__ out, long long m) {
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < m; i += (long long)gridDim.x * kThreads)
    out[i] = (TO)in[i];
}

// F = I on every voxel (the stress-free start of Algorithm 1).
__global__ __launch_bounds__(kThreads) void k_set_identity(Batch B, double* __restrict__ F) {
  int local;
  const int rv = find_rve(B, K_VOX, blockIdx.x, local);
  const Grid& g = B.grids[rv];
  const int nb = rve_blocks(B, K_VOX, rv);
  const long long n = g.n, off = 9 * g.vox_off;
  FOR_RVE_RANGE(v, n, local, nb) {
#pragma unroll
    for (int c = 0; c < 9; ++c) F[off + c * n + v] = (c % 4 == 0) ? 1.0 : 0.0;
  }
}

// Adjoint gradient per voxel at the converged F with adjoint field w and the
// RVE's cotangent g (Batch::uni):
//   dL/dmu = (1/n) (g - w) : F . 2 dev(E),  dL/dK = (1/n) (g - w) : tr(E) F
// (S = (K - 2mu/3) tr(E) I + 2 mu E).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_adjoint_grad(Batch B, const double* __restrict__ F,
                                                           const T* __restrict__ w, double* __restrict__ dmu,
                                                           double* __restrict__ dK) {
  int local;
  const int rv = find_rve(B, K_VOX, blockIdx.x, local);
  if (skip_rve(B, nullptr, rv)) return;
  const Grid& g = B.grids[rv];
  const int nb = rve_blocks(B, K_VOX, rv);
  const long long n = g.n, off = 9 * g.vox_off;
  const double* gb = B.uni + 9 * rv;
  FOR_RVE_RANGE(v, n, local, nb) {
    double f[9], d[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      f[c] = F[off + c * n + v];
      d[c] = gb[c] - (double)w[off + c * n + v];
    }
    double C[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) C[3 * i + j] = f[i] * f[j] + f[3 + i] * f[3 + j] + f[6 + i] * f[6 + j];
    const double trE = 0.5 * (C[0] + C[4] + C[8] - 3.0);
    double D[9];  // 2 dev E = C - I - (2/3) tr(E) I
#pragma unroll
    for (int c = 0; c < 9; ++c) D[c] = C[c];
    D[0] -= 1.0 + 2.0 * trE / 3.0;
    D[4] -= 1.0 + 2.0 * trE / 3.0;
    D[8] -= 1.0 + 2.0 * trE / 3.0;
    double Q[9];
    mat33<double>(f, D, Q);
    double smu = 0.0, sK = 0.0;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      smu += d[c] * Q[c];
      sK += d[c] * f[c];
    }
    dmu[g.vox_off + v] = smu * g.inv_n;
    if (dK) dK[g.vox_off + v] = sK * trE * g.inv_n;
  }
}

// Column of the macroscopic tangent: the sums over the cell of K(F) : (U - w)
// with U the RVE's uniform tensor (a unit macroscopic increment) and w the
// solution of A w = G(K(F) : U); into SLOT_PBAR .. SLOT_PBAR + 8.
template <int LAW>
__global__ __launch_bounds__(kThreads) void k_tangent_sum(Batch B, Material mat, const double* __restrict__ F,
                                                          const double* __restrict__ w) {
  int local;
  const int rv = find_rve(B, K_VOX, blockIdx.x, local);
  if (skip_rve(B, nullptr, rv)) return;
  const Grid& g = B.grids[rv];
  const int nb = rve_blocks(B, K_VOX, rv);
  const long long n = g.n, off = 9 * g.vox_off;
  const double* u = B.uni + 9 * rv;
  double acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = 0.0;
  FOR_RVE_RANGE(v, n, local, nb) {
    double f[9], q[9], d[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      f[c] = F[off + c * n + v];
      q[c] = u[c] - w[off + c * n + v];
    }
    if constexpr (LAW == MODEL_J2) {
      double K, mu, ty0, H, h[7];
      j2_point_data(mat, g.vox_off + v, K, mu, ty0, H, h);
      j2_tangent(f, h, K, mu, ty0, H, q, d);
    } else {
      double lam, mu;
      material_at(mat, g.vox_off + v, lam, mu);
      svk_tangent<double>(f, q, lam, mu, d);
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) acc[c] += d[c];
  }
  double res[9];
  block_sums<9>(acc, res);
  if (threadIdx.x == 0)
    for (int c = 0; c < 9; ++c) pslot(B, SLOT_PBAR + c)[blockIdx.x] = res[c];
}

// ---------------------------------------------------------------------------
// GMRES building blocks (Arnoldi with classical Gram-Schmidt).  Each cell's
// 9 n values are taken in element pairs, one 2-element vector load per field
// (the basis stride is even and every field starts on a 256-byte boundary):
// pairs start at the first even global index of the cell; the one or two
// elements left over at the cell's ends go to the first thread of the cell's
// first work-group.
// ---------------------------------------------------------------------------
template <typename T>
struct Pair2;
template <>
struct Pair2<double> { using type = double2; };
template <>
struct Pair2<float> { using type = float2; };

struct PairRange {
  long long s0, np, lone[2];
  int nlone;
  __device__ PairRange(long long off, long long m) {
    s0 = off & 1;
    np = (m - s0) >> 1;
    nlone = 0;
    if (s0 && m > 0) lone[nlone++] = 0;
    if (m > s0 && ((m - s0) & 1)) lone[nlone++] = m - 1;
  }
};

// K (1..kGmDot) is the number of basis vectors of the launch, fixed at
// compile time so that all K loads of an element pair are issued before the
// first is used.
template <typename T, int K>
__global__ __launch_bounds__(kThreads) void k_gm_dots(Batch B, const T* __restrict__ w, const T* __restrict__ V,
                                                      long long vstride, int i0, int ww) {
  using P2 = typename Pair2<T>::type;
  int local;
  const int rv = find_rve(B, K_ELEM9, blockIdx.x, local);
  if (skip_rve(B, nullptr, rv)) return;
  const Grid& g = B.grids[rv];
  const int nb = rve_blocks(B, K_ELEM9, rv);
  const long long m = 9 * g.n, off = 9 * g.vox_off;
  const PairRange pr(off, m);
  const T* Vq = V + (long long)i0 * vstride + off;
  const T* wc = w + off;
  double acc[K + 1];
#pragma unroll
  for (int q = 0; q <= K; ++q) acc[q] = 0.0;
  FOR_RVE_RANGE(p, pr.np, local, nb) {
    const long long e = pr.s0 + 2 * p;
    const P2 wv = *reinterpret_cast<const P2*>(wc + e);
    P2 v[K];
#pragma unroll
    for (int q = 0; q < K; ++q) v[q] = *reinterpret_cast<const P2*>(Vq + q * vstride + e);
#pragma unroll
    for (int q = 0; q < K; ++q) acc[q] += (double)wv.x * (double)v[q].x + (double)wv.y * (double)v[q].y;
    acc[K] += (double)wv.x * (double)wv.x + (double)wv.y * (double)wv.y;
  }
  if (local == 0 && threadIdx.x == 0)
    for (int t = 0; t < pr.nlone; ++t) {
      const long long e = pr.lone[t];
      const double wi = (double)wc[e];
#pragma unroll
      for (int q = 0; q < K; ++q) acc[q] += wi * (double)Vq[q * vstride + e];
      acc[K] += wi * wi;
    }
  double res[K + 1];
  block_sums<K + 1>(acc, res);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < K; ++q) pslot(B, SLOT_DOT + q)[blockIdx.x] = res[q];
    if (ww) pslot(B, SLOT_AUX)[blockIdx.x] = res[K];  // ||w||^2
  }
}

// y += sum_q coef[rv][q] V_{i0+q}; with norm ||y||^2 into SLOT_RR; with DOTS
// also <y, V_{i0+q}> of the updated y into SLOT_DOT + q (the next Gram-Schmidt
// pass's inner products, from the basis values already loaded).
template <typename T, int K, bool DOTS>
__global__ __launch_bounds__(kThreads) void k_gm_update(Batch B, T* __restrict__ y, const T* __restrict__ V,
                                                        long long vstride, int i0,
                                                        const double* __restrict__ coef, int norm) {
  using P2 = typename Pair2<T>::type;
  int local;
  const int rv = find_rve(B, K_ELEM9, blockIdx.x, local);
  if (skip_rve(B, nullptr, rv)) return;
  const Grid& g = B.grids[rv];
  const int nb = rve_blocks(B, K_ELEM9, rv);
  const long long m = 9 * g.n, off = 9 * g.vox_off;
  const PairRange pr(off, m);
  const T* Vq = V + (long long)i0 * vstride + off;
  T* yc = y + off;
  double c[K];
#pragma unroll
  for (int q = 0; q < K; ++q) c[q] = coef[rv * kGmCoef + q];
  constexpr int NA = DOTS ? K + 1 : 1;  // [dots..., ||y||^2]
  double acc[NA];
#pragma unroll
  for (int q = 0; q < NA; ++q) acc[q] = 0.0;
  FOR_RVE_RANGE(p, pr.np, local, nb) {
    const long long e = pr.s0 + 2 * p;
    const P2 yv = *reinterpret_cast<const P2*>(yc + e);
    P2 a[K];
#pragma unroll
    for (int q = 0; q < K; ++q) a[q] = *reinterpret_cast<const P2*>(Vq + q * vstride + e);
    double v0 = (double)yv.x, v1 = (double)yv.y;
#pragma unroll
    for (int q = 0; q < K; ++q) {
      v0 += c[q] * (double)a[q].x;
      v1 += c[q] * (double)a[q].y;
    }
    P2 t;
    t.x = (T)v0;
    t.y = (T)v1;
    *reinterpret_cast<P2*>(yc + e) = t;
    if constexpr (DOTS) {
#pragma unroll
      for (int q = 0; q < K; ++q) acc[q] += (double)t.x * (double)a[q].x + (double)t.y * (double)a[q].y;
    }
    acc[NA - 1] += (double)t.x * (double)t.x + (double)t.y * (double)t.y;
  }
  if (local == 0 && threadIdx.x == 0)
    for (int u = 0; u < pr.nlone; ++u) {
      const long long e = pr.lone[u];
      double v = (double)yc[e];
#pragma unroll
      for (int q = 0; q < K; ++q) v += c[q] * (double)Vq[q * vstride + e];
      const T t = (T)v;
      yc[e] = t;
      if constexpr (DOTS) {
#pragma unroll
        for (int q = 0; q < K; ++q) acc[q] += (double)t * (double)Vq[q * vstride + e];
      }
      acc[NA - 1] += (double)t * (double)t;
    }
  if (norm || DOTS) {
    double res[NA];
    block_sums<NA>(acc, res);
    if (threadIdx.x == 0) {
      if constexpr (DOTS) {
#pragma unroll
        for (int q = 0; q < K; ++q) pslot(B, SLOT_DOT + q)[blockIdx.x] = res[q];
      }
      pslot(B, SLOT_RR)[blockIdx.x] = res[NA - 1];
    }
  }
}

// dst may alias s1 (an in-place scaling): no restrict on those two
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gm_lincomb(Batch B, T* dst, const T* s1, const T* __restrict__ s2,
                                                         const double* __restrict__ coef, int norm) {
  using P2 = typename Pair2<T>::type;
  int local;
  const int rv = find_rve(B, K_ELEM9, blockIdx.x, local);
  if (skip_rve(B, nullptr, rv)) return;
  const Grid& g = B.grids[rv];
  const int nb = rve_blocks(B, K_ELEM9, rv);
  const long long m = 9 * g.n, off = 9 * g.vox_off;
  const PairRange pr(off, m);
  const double a = coef[rv * kGmCoef], b = coef[rv * kGmCoef + 1];
  T* dc = dst + off;
  const T* c1 = s1 + off;
  const T* c2 = s2 ? s2 + off : nullptr;
  double acc[1] = {0.0};
  FOR_RVE_RANGE(p, pr.np, local, nb) {
    const long long e = pr.s0 + 2 * p;
    const P2 u = *reinterpret_cast<const P2*>(c1 + e);
    double v0 = a * (double)u.x, v1 = a * (double)u.y;
    if (c2) {
      const P2 u2 = *reinterpret_cast<const P2*>(c2 + e);
      v0 += b * (double)u2.x;
      v1 += b * (double)u2.y;
    }
    P2 t;
    t.x = (T)v0;
    t.y = (T)v1;
    *reinterpret_cast<P2*>(dc + e) = t;
    acc[0] += (double)t.x * (double)t.x + (double)t.y * (double)t.y;
  }
  if (local == 0 && threadIdx.x == 0)
    for (int u = 0; u < pr.nlone; ++u) {
      const long long e = pr.lone[u];
      double v = a * (double)c1[e];
      if (c2) v += b * (double)c2[e];
      const T t = (T)v;
      dc[e] = t;
      acc[0] += (double)t * (double)t;
    }
  if (norm) {
    double res[1];
    block_sums<1>(acc, res);
    if (threadIdx.x == 0) pslot(B, SLOT_RR)[blockIdx.x] = res[0];
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_cg_finish(int prec, const Launch& L, void* x, const void* p, const CgState* cg) {
  const dim3 grid(L.nblk[K_ELEM9]), block(kThreads);
  if (prec == PREC_F64)
    hipLaunchKernelGGL((k_cg_finish<double>), grid, block, 0, L.s, L.b, static_cast<double*>(x),
                       static_cast<const double*>(p), cg);
  else
    hipLaunchKernelGGL((k_cg_finish<float>), grid, block, 0, L.s, L.b, static_cast<float*>(x),
                       static_cast<const float*>(p), cg);
}

void launch_cg_beta(const Launch& L, CgState* cg) {
  hipLaunchKernelGGL(k_cg_beta, dim3(L.b.nrve), dim3(kThreads), 0, L.s, L.b, cg);
}

void launch_cg_init(const Launch& L, CgState* cg, double eta, int max_cg, int stall, int method, double lo,
                    double hi) {
  hipLaunchKernelGGL(k_cg_init, dim3(L.b.nrve), dim3(kThreads), 0, L.s, L.b, cg, eta, max_cg, stall, method, lo, hi);
}

void launch_set_F(const Launch& L, const double* Ft, double* F, float* Flin32) {
  hipLaunchKernelGGL(k_set_F, dim3(L.nblk[K_VOX]), dim3(kThreads), 0, L.s, L.b, Ft, F, Flin32);
}

void launch_newton_update(int prec, const Launch& L, const Material& mat, double* F, const void* x, double* P,
                          float* Flin32, bool add_uni) {
  const dim3 grid(L.nblk[K_VOX]), block(kThreads);
  if (mat.model == MODEL_J2)
    hipLaunchKernelGGL((k_newton_update<double, MODEL_J2>), grid, block, 0, L.s, L.b, mat, F,
                       static_cast<const double*>(x), P, Flin32, add_uni ? 1 : 0);
  else if (prec == PREC_F64)
    hipLaunchKernelGGL((k_newton_update<double, MODEL_SVK>), grid, block, 0, L.s, L.b, mat, F,
                       static_cast<const double*>(x), P, Flin32, add_uni ? 1 : 0);
  else
    hipLaunchKernelGGL((k_newton_update<float, MODEL_SVK>), grid, block, 0, L.s, L.b, mat, F,
                       static_cast<const float*>(x), P, Flin32, add_uni ? 1 : 0);
}

void launch_constitutive(const Launch& L, const Material& mat, const double* F, double* P) {
  if (mat.model == MODEL_J2)
    hipLaunchKernelGGL((k_constitutive<MODEL_J2>), dim3(L.nblk[K_VOX]), dim3(kThreads), 0, L.s, L.b, mat, F, P);
  else
    hipLaunchKernelGGL((k_constitutive<MODEL_SVK>), dim3(L.nblk[K_VOX]), dim3(kThreads), 0, L.s, L.b, mat, F, P);
}

// The compact J2 tangent at the linearisation point F (committed history).
__global__ __launch_bounds__(kThreads) void k_j2_tangent_data(Batch B, Material mat, const double* __restrict__ F,
                                                             double* __restrict__ out) {
  int local;
  const int rv = find_rve(B, K_VOX, blockIdx.x, local);
  if (skip_rve(B, nullptr, rv)) return;
  const Grid& g = B.grids[rv];
  const int nb = rve_blocks(B, K_VOX, rv);
  const long long n = g.n, off = 9 * g.vox_off;
  FOR_RVE_RANGE(v, n, local, nb) {
    double f[9], t[kJ2Tan], K, mu, ty0, H, h[7];
#pragma unroll
    for (int c = 0; c < 9; ++c) f[c] = F[off + c * n + v];
    const long long gv = g.vox_off + v;
    j2_point_data(mat, gv, K, mu, ty0, H, h);
    j2_tangent_data(f, h, K, mu, ty0, H, t);
#pragma unroll
    for (int k = 0; k < kJ2Tan; ++k) out[k * mat.ntot + gv] = t[k];
  }
}

void launch_j2_tangent_data(const Launch& L, const Material& mat, const double* F, double* out) {
  hipLaunchKernelGGL(k_j2_tangent_data, dim3(L.nblk[K_VOX]), dim3(kThreads), 0, L.s, L.b, mat, F, out);
}

// J2 virgin state: Cp^-1 = I, eps_p = 0 ([7][ntot])
__global__ __launch_bounds__(kThreads) void k_virgin_history(double* __restrict__ h, long long ntot) {
  for (long long v = blockIdx.x * (long long)kThreads + threadIdx.x; v < ntot; v += (long long)gridDim.x * kThreads)
#pragma unroll
    for (int k = 0; k < 7; ++k) h[k * ntot + v] = k < 3 ? 1.0 : 0.0;
}

void launch_set_virgin_history(const Launch& L, double* hist, long long ntot) {
  hipLaunchKernelGGL(k_virgin_history, dim3(elem_blocks(ntot)), dim3(kThreads), 0, L.s, hist, ntot);
}

void launch_field_sum(const Launch& L, const double* X, int slot0) {
  hipLaunchKernelGGL(k_field_sum, dim3(L.nblk[K_VOX]), dim3(kThreads), 0, L.s, L.b, X, slot0);
}

void launch_reduce(const Launch& L, int kind, int slot0, int nslots, double* out) {
  hipLaunchKernelGGL(k_reduce, dim3(L.b.nrve, nslots), dim3(kThreads), 0, L.s, L.b, kind, slot0, out);
}

void launch_convert(int to_prec, const void* in, void* out, long long count, hipStream_t s) {
  const int nb = elem_blocks(count);
  if (to_prec == PREC_F32)
    hipLaunchKernelGGL((k_convert<double, float>), dim3(nb), dim3(kThreads), 0, s, static_cast<const double*>(in),
                       static_cast<float*>(out), count);
  else
    hipLaunchKernelGGL((k_convert<float, double>), dim3(nb), dim3(kThreads), 0, s, static_cast<const float*>(in),
                       static_cast<double*>(out), count);
}

void launch_set_identity(const Launch& L, double* F) {
  hipLaunchKernelGGL(k_set_identity, dim3(L.nblk[K_VOX]), dim3(kThreads), 0, L.s, L.b, F);
}

// the launch with K = k, for k in 1..kGmDot
template <typename F, int... Ks>
void with_k(int k, F&& f, std::integer_sequence<int, Ks...>) {
  ((k == Ks + 1 ? f(std::integral_constant<int, Ks + 1>{}) : void()), ...);
}

void launch_gm_dots(int prec, const Launch& L, const void* w, const void* V, long long vstride, int i0, int k,
                    bool ww) {
  const dim3 grid(L.nblk[K_ELEM9]), block(kThreads);
  with_k(k, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    if (prec == PREC_F64)
      hipLaunchKernelGGL((k_gm_dots<double, K>), grid, block, 0, L.s, L.b, static_cast<const double*>(w),
                         static_cast<const double*>(V), vstride, i0, ww ? 1 : 0);
    else
      hipLaunchKernelGGL((k_gm_dots<float, K>), grid, block, 0, L.s, L.b, static_cast<const float*>(w),
                         static_cast<const float*>(V), vstride, i0, ww ? 1 : 0);
  }, std::make_integer_sequence<int, kGmDot>{});
}

void launch_gm_update(int prec, const Launch& L, void* y, const void* V, long long vstride, int i0, int k,
                      const double* coef, bool norm, bool dots) {
  const dim3 grid(L.nblk[K_ELEM9]), block(kThreads);
  with_k(k, [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    if (prec == PREC_F64) {
      double* yy = static_cast<double*>(y);
      const double* vv = static_cast<const double*>(V);
      if (dots)
        hipLaunchKernelGGL((k_gm_update<double, K, true>), grid, block, 0, L.s, L.b, yy, vv, vstride, i0, coef, 1);
      else
        hipLaunchKernelGGL((k_gm_update<double, K, false>), grid, block, 0, L.s, L.b, yy, vv, vstride, i0, coef,
                           norm ? 1 : 0);
    } else {
      float* yy = static_cast<float*>(y);
      const float* vv = static_cast<const float*>(V);
      if (dots)
        hipLaunchKernelGGL((k_gm_update<float, K, true>), grid, block, 0, L.s, L.b, yy, vv, vstride, i0, coef, 1);
      else
        hipLaunchKernelGGL((k_gm_update<float, K, false>), grid, block, 0, L.s, L.b, yy, vv, vstride, i0, coef,
                           norm ? 1 : 0);
    }
  }, std::make_integer_sequence<int, kGmDot>{});
}

void launch_gm_lincomb(int prec, const Launch& L, void* dst, const void* s1, const void* s2, const double* coef,
                       bool norm) {
  const dim3 grid(L.nblk[K_ELEM9]), block(kThreads);
  if (prec == PREC_F64)
    hipLaunchKernelGGL((k_gm_lincomb<double>), grid, block, 0, L.s, L.b, static_cast<double*>(dst),
                       static_cast<const double*>(s1), static_cast<const double*>(s2), coef, norm ? 1 : 0);
  else
    hipLaunchKernelGGL((k_gm_lincomb<float>), grid, block, 0, L.s, L.b, static_cast<float*>(dst),
                       static_cast<const float*>(s1), static_cast<const float*>(s2), coef, norm ? 1 : 0);
}

void launch_tangent_sum(const Launch& L, const Material& mat, const double* F, const double* w) {
  if (mat.model == MODEL_J2)
    hipLaunchKernelGGL((k_tangent_sum<MODEL_J2>), dim3(L.nblk[K_VOX]), dim3(kThreads), 0, L.s, L.b, mat, F, w);
  else
    hipLaunchKernelGGL((k_tangent_sum<MODEL_SVK>), dim3(L.nblk[K_VOX]), dim3(kThreads), 0, L.s, L.b, mat, F, w);
}

void launch_adjoint_grad(int prec, const Launch& L, const double* F, const void* w, double* dmu, double* dK) {
  const dim3 grid(L.nblk[K_VOX]), block(kThreads);
  if (prec == PREC_F64)
    hipLaunchKernelGGL((k_adjoint_grad<double>), grid, block, 0, L.s, L.b, F, static_cast<const double*>(w), dmu, dK);
  else
    hipLaunchKernelGGL((k_adjoint_grad<float>), grid, block, 0, L.s, L.b, F, static_cast<const float*>(w), dmu, dK);
}

}  // namespace fftnk
