// The five passes of the projected-tangent operator of the finite-strain FFT
// Newton-Krylov method (de Geus et al. 2017, Sec. 2.5-2.6): A p = G(K(F) : p).
//   pass 1  tangent action K(F) : p per voxel (Sec. 4.3) + a2 real-to-complex DFT
//   pass 2  a1 forward DFT
//   pass 3  a0 forward DFT, projection G-hat, a0 inverse DFT
//   pass 4  a1 inverse DFT
//   pass 5  a2 complex-to-real inverse DFT (+ CG partial sums)
// Every launch covers all RVEs of a context (work-group -> RVE through the
// launch kind's start table).  Power-of-two a1 / a0 axes use the register-
// resident engine; everything else the LDS Stockham engine.
#include "fftnk_device.h"
#include "fftnk_j2.h"

namespace fftnk {

// ---------------------------------------------------------------------------
// launch geometry
// ---------------------------------------------------------------------------
int elem_blocks(long long m) {
  long long b = (m + kThreads - 1) / kThreads;
  if (b > kRedBlocks) b = kRedBlocks;
  if (b < 1) b = 1;
  return (int)b;
}

int row_blocks(const Grid& g) { return (int)((g.rows + g.rt - 1) / g.rt); }

static int reg_pencils(int n) { return kThreads / (n / kRegP); }  // pencils per work-group, register engine

int col1_blocks(const Grid& g, int prec) {
  if (g.ax[1].reg) {
    const long long np = 9LL * g.n0 * g.h, mb = reg_pencils(g.n1);
    return (int)((np + mb - 1) / mb);
  }
  const int M = prec == PREC_F64 ? g.m64 : g.m32;
  return 9 * g.n0 * ((g.h + M - 1) / M);
}

int col0_blocks(const Grid& g, int prec) {
  if (g.ax[0].reg) {
    const long long np = 3LL * g.n1 * g.h, mb = reg_pencils(g.n0);
    return (int)((np + mb - 1) / mb);
  }
  const int M = prec == PREC_F64 ? g.m64 : g.m32;
  return 3 * g.n1 * ((g.h + M - 1) / M);
}

// ---------------------------------------------------------------------------
// Pass 1: a2 forward transform of the 9 components, fused with the production
// of the field being transformed.  Each work-group owns g.rt consecutive grid
// lines.  Component pairs (0,1) (2,3) (4,5) (6,7) are packed as x + i y into
// one complex transform (two real transforms for the price of one), component
// 8 rides alone; the half spectra are unpacked with X[k] = (Z[k] + conj Z[-k])/2
// and Y[k] = (Z[k] - conj Z[-k]) / (2i).
// ---------------------------------------------------------------------------
// Tangent action of the voxel's material law at F on the direction p.
template <typename T, int LAW>
__device__ __forceinline__ void tangent_at(const Material& mat, long long gv, const T* F, const T* p, T* d) {
  if constexpr (LAW == MODEL_J2) {
    double K, mu, ty0, H, h[7];
    j2_point_data(mat, gv, K, mu, ty0, H, h);
    j2_tangent(F, h, K, mu, ty0, H, p, d);
  } else {
    double lam, mu;
    material_at(mat, gv, lam, mu);
    svk_tangent<T>(F, p, (T)lam, (T)mu, d);
  }
}

template <typename T, int MODE, int LAW>
__global__ __launch_bounds__(kThreads) void k_fwd_a2(Batch B, Material mat, const T* __restrict__ in,
                                                     const T* __restrict__ rvec, T* __restrict__ pvec,
                                                     const T* __restrict__ Flin, double scale,
                                                     cx<T>* __restrict__ spec, const CgState* __restrict__ cg) {
  int local;
  const int rv = find_rve(B, K_ROW, blockIdx.x, local);
  if (skip_rve(B, MODE == FWD_CG ? cg : nullptr, rv)) return;
  const Grid& g = B.grids[rv];
  extern __shared__ unsigned char smem_raw[];
  const int N2 = g.n2, RT = g.rt, H = g.h;
  const int npen = 5 * RT;
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* bufA = tw + N2;
  cx<T>* bufB = bufA + npen * N2;
  load_twiddles<T>(tw, B, g.ax[2].tw, N2);

  const long long n = g.n;
  const long long off = 9 * g.vox_off;
  const long long row0 = (long long)local * RT;
  double beta = 0.0;
  bool first = false;
  if (MODE == FWD_CG) {
    beta = cg[rv].beta;
    first = cg[rv].iter == 0;
  }
  double acc[1] = {0.0};
  // register engine: pencil slot m = pair * RT + line (slots >= 5 RT idle),
  // stage the field in LDS once, transform in registers, unpack through one
  // mirror exchange.  bufA holds one slot of N2 entries per kThreads / Tp.
  const bool reg = g.ax[2].reg;
  for (int t = threadIdx.x; t < RT * N2; t += kThreads) {
    const int rl = t / N2, a2 = t - rl * N2;
    const long long row = row0 + rl;
    T d[9];
    if (row < g.rows) {
      const long long v = row * N2 + a2;
      if (MODE == FWD_COPY) {
#pragma unroll
        for (int c = 0; c < 9; ++c) d[c] = (T)scale * in[off + c * n + v];
      } else {
        T p[9], F[9];
        if (MODE == FWD_TANGENT_UNI) {
#pragma unroll
          for (int c = 0; c < 9; ++c) p[c] = (T)B.uni[9 * rv + c];
        } else if (MODE == FWD_TANGENT) {
#pragma unroll
          for (int c = 0; c < 9; ++c) p[c] = in[off + c * n + v];
        } else {  // FWD_CG
#pragma unroll
          for (int c = 0; c < 9; ++c) {
            const T r = rvec[off + c * n + v];
            p[c] = first ? r : r + (T)beta * pvec[off + c * n + v];
            pvec[off + c * n + v] = p[c];
          }
        }
#pragma unroll
        for (int c = 0; c < 9; ++c) F[c] = Flin[off + c * n + v];
        tangent_at<T, LAW>(mat, g.vox_off + v, F, p, d);
      }
#pragma unroll
      for (int c = 0; c < 9; ++c) acc[0] += (double)d[c] * (double)d[c];
    } else {
#pragma unroll
      for (int c = 0; c < 9; ++c) d[c] = (T)0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) bufA[(q * RT + rl) * N2 + a2] = cx<T>{d[2 * q], d[2 * q + 1]};
    bufA[(4 * RT + rl) * N2 + a2] = cx<T>{d[8], (T)0};
  }
  __syncthreads();
  const long long srow = g.rows * H;
  cx<T>* S = spec + g.spec_off;

  if (reg) {
    const int Tp = N2 / kRegP;
    const int m = threadIdx.x / Tp, t = threadIdx.x - m * Tp;
    cx<T>* xl = bufA + m * N2;
    cx<T> v[kRegP];
#pragma unroll
    for (int q = 0; q < kRegP; ++q) v[q] = xl[t + Tp * q];
    __syncthreads();
    reg_fft<T>(v, g.ax[2], t, Tp, tw, false, xl, 1);
#pragma unroll
    for (int q = 0; q < kRegP; ++q) xl[t + Tp * q] = v[q];
    __syncthreads();
    const int pq = m / RT, rl = m - pq * RT;
    const long long row = row0 + rl;
    if (m < npen && row < g.rows) {
#pragma unroll
      for (int q = 0; q < kRegP / 2; ++q) {  // k = t + Tp q < n2 / 2 = h
        const int k = t + Tp * q;
        const cx<T> z = v[q];
        const cx<T> zm = xl[k ? N2 - k : 0];
        if (pq == 4) {
          S[8 * srow + row * H + k] = z;
        } else {
          S[(2 * pq) * srow + row * H + k] = cx<T>{(T)0.5 * (z.x + zm.x), (T)0.5 * (z.y - zm.y)};
          S[(2 * pq + 1) * srow + row * H + k] = cx<T>{(T)0.5 * (z.y + zm.y), (T)-0.5 * (z.x - zm.x)};
        }
      }
    }
    if (MODE != FWD_CG) {
      double res[1];
      block_sums<1>(acc, res);
      if (threadIdx.x == 0) pslot(B, SLOT_YY)[blockIdx.x] = res[0];
    }
    return;
  }

  const cx<T>* Z = fft_lds<T>(bufA, bufB, g.ax[2], npen, N2, 1, tw, false, false);
  for (int t = threadIdx.x; t < 9 * RT * H; t += kThreads) {
    const int c = t / (RT * H);
    const int rem = t - c * RT * H;
    const int rl = rem / H, k = rem - rl * H;
    const long long row = row0 + rl;
    if (row >= g.rows) continue;
    const int pen = (c >> 1) * RT + rl;
    const cx<T> z = Z[pen * N2 + k];
    const cx<T> zm = Z[pen * N2 + (k ? N2 - k : 0)];
    cx<T> o;
    if (c == 8) {
      o = z;
    } else if ((c & 1) == 0) {
      o = cx<T>{(T)0.5 * (z.x + zm.x), (T)0.5 * (z.y - zm.y)};
    } else {
      o = cx<T>{(T)0.5 * (z.y + zm.y), (T)-0.5 * (z.x - zm.x)};
    }
    S[c * srow + row * H + k] = o;
  }
  if (MODE != FWD_CG) {
    double res[1];
    block_sums<1>(acc, res);
    if (threadIdx.x == 0) pslot(B, SLOT_YY)[blockIdx.x] = res[0];
  }
}

// ---------------------------------------------------------------------------
// Pass 2 / 4: transform along a1 (forward or inverse) in place.
// Register engine: kThreads / (n1/8) pencils per work-group, consecutive in
// (component, a0, k2) order so that each load / store row of the work-group is
// a run of consecutive k2.  LDS engine: g.m consecutive k2 of one
// (component, a0) plane.
// ---------------------------------------------------------------------------
template <typename T, bool INV>
__global__ __launch_bounds__(kThreads) void k_col_a1(Batch B, cx<T>* __restrict__ spec,
                                                     const CgState* __restrict__ cg) {
  int local;
  const int rv = find_rve(B, sizeof(T) == 8 ? K_COL1_64 : K_COL1_32, blockIdx.x, local);
  if (skip_rve(B, cg, rv)) return;
  const Grid& g = B.grids[rv];
  extern __shared__ unsigned char smem_raw[];
  const int N1 = g.n1, H = g.h;
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  load_twiddles<T>(tw, B, g.ax[1].tw, N1);
  cx<T>* S0 = spec + g.spec_off;

  if (g.ax[1].reg) {
    cx<T>* xl = tw + N1;
    const int Tp = N1 / kRegP, Mb = kThreads / Tp;
    const int m = threadIdx.x % Mb, t = threadIdx.x / Mb;
    const long long npen = 9LL * g.n0 * H;
    long long pen = (long long)local * Mb + m;
    const bool valid = pen < npen;
    if (!valid) pen = 0;
    const long long plane = pen / H;
    cx<T>* base = S0 + plane * N1 * H + (pen - plane * H);
    cx<T> v[kRegP];
#pragma unroll
    for (int q = 0; q < kRegP; ++q) v[q] = valid ? base[(long long)(t + Tp * q) * H] : cx<T>{(T)0, (T)0};
    reg_fft<T>(v, g.ax[1], t, Tp, tw, INV, xl + m, Mb);
    if (valid) {
#pragma unroll
      for (int q = 0; q < kRegP; ++q) base[(long long)(t + Tp * q) * H] = v[q];
    }
    return;
  }

  const int M = sizeof(T) == 8 ? g.m64 : g.m32;
  cx<T>* bufA = tw + N1;
  cx<T>* bufB = bufA + N1 * M;
  const int nkb = (H + M - 1) / M;
  const int c = local / (g.n0 * nkb);
  const int rem = local - c * g.n0 * nkb;
  const int a0 = rem / nkb, kb = rem - a0 * nkb;
  const int Mt = min(M, H - kb * M);
  cx<T>* base = S0 + (long long)c * g.rows * H + (long long)a0 * N1 * H + kb * M;
  for (int t = threadIdx.x; t < N1 * M; t += kThreads) {
    const int e = t / M, m = t - e * M;
    bufA[t] = m < Mt ? base[(long long)e * H + m] : cx<T>{(T)0, (T)0};
  }
  __syncthreads();
  const cx<T>* R = fft_lds<T>(bufA, bufB, g.ax[1], M, 1, M, tw, INV, true);
  for (int t = threadIdx.x; t < N1 * M; t += kThreads) {
    const int e = t / M, m = t - e * M;
    if (m < Mt) base[(long long)e * H + m] = R[t];
  }
}

// ---------------------------------------------------------------------------
// Pass 3: a0 forward transform, projection, a0 inverse transform.  A pencil is
// one (tensor row i, k1, k2) triple carrying the three components 3i..3i+2:
// G-hat_ijlm = delta_im g_jl (App. D), so row i of the projected field needs
// row i of the input only.  G-hat (Sec. 2.5; App. C for even axes):
//   out_ij = xi_j (sum_l xi_l A_il) / |xi|^2 / n,   xi_d = k_d / N_d,
// zero at k = 0 and whenever an even axis sits at its Nyquist index.  The 1/n
// of the inverse transform is folded in here.
// ---------------------------------------------------------------------------
constexpr int kMaxPpt = 8;  // points per thread of an LDS-engine pass-3 tile (n0 * m <= kMaxPpt * kThreads)

template <typename T>
__device__ __forceinline__ void project_point(cx<T>& a0, cx<T>& a1, cx<T>& a2, int k0, int k1, int k2,
                                              const Grid& g) {
  const int f0 = signed_freq(k0, g.n0), f1 = signed_freq(k1, g.n1);
  const bool zero = (f0 == 0 && f1 == 0 && k2 == 0) || ((g.n0 % 2 == 0) && (2 * k0 == g.n0)) ||
                    ((g.n1 % 2 == 0) && (2 * k1 == g.n1));
  if (zero) {
    a0 = a1 = a2 = cx<T>{(T)0, (T)0};
    return;
  }
  const T xi0 = (T)f0 / (T)g.n0, xi1 = (T)f1 / (T)g.n1, xi2 = (T)k2 / (T)g.n2;
  const T coef = (T)g.inv_n / (xi0 * xi0 + xi1 * xi1 + xi2 * xi2);
  cx<T> s = cscale(a0, xi0);
  s = s + cscale(a1, xi1);
  s = s + cscale(a2, xi2);
  a0 = cscale(s, xi0 * coef);
  a1 = cscale(s, xi1 * coef);
  a2 = cscale(s, xi2 * coef);
}

template <typename T>
__global__ __launch_bounds__(kThreads, 3) void k_col_a0_project(Batch B, cx<T>* __restrict__ spec,
                                                             const CgState* __restrict__ cg) {
  int local;
  const int rv = find_rve(B, sizeof(T) == 8 ? K_COL0_64 : K_COL0_32, blockIdx.x, local);
  if (skip_rve(B, cg, rv)) return;
  const Grid& g = B.grids[rv];
  extern __shared__ unsigned char smem_raw[];
  const int N0 = g.n0, N1 = g.n1, H = g.h;
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  load_twiddles<T>(tw, B, g.ax[0].tw, N0);
  cx<T>* S0 = spec + g.spec_off;
  const long long S = (long long)N1 * H;  // element stride along a0
  const long long cstride = g.rows * H;

  if (g.ax[0].reg) {
    cx<T>* xl = tw + N0;
    const int Tp = N0 / kRegP, Mb = kThreads / Tp;
    const int m = threadIdx.x % Mb, t = threadIdx.x / Mb;
    const long long npen = 3LL * N1 * H;
    long long pen = (long long)local * Mb + m;
    const bool valid = pen < npen;
    if (!valid) pen = 0;
    const long long qq = pen / H;
    const int k2 = (int)(pen - qq * H);
    const int i = (int)(qq / N1), k1 = (int)(qq - (long long)i * N1);
    cx<T>* base = S0 + (long long)(3 * i) * cstride + (long long)k1 * H + k2;
    cx<T> v0[kRegP], v1[kRegP], v2[kRegP];
#pragma unroll
    for (int q = 0; q < kRegP; ++q) {
      const long long e = (long long)(t + Tp * q) * S;
      v0[q] = valid ? base[e] : cx<T>{(T)0, (T)0};
      v1[q] = valid ? base[cstride + e] : cx<T>{(T)0, (T)0};
      v2[q] = valid ? base[2 * cstride + e] : cx<T>{(T)0, (T)0};
    }
    reg_fft<T>(v0, g.ax[0], t, Tp, tw, false, xl + m, Mb);
    reg_fft<T>(v1, g.ax[0], t, Tp, tw, false, xl + m, Mb);
    reg_fft<T>(v2, g.ax[0], t, Tp, tw, false, xl + m, Mb);
#pragma unroll
    for (int q = 0; q < kRegP; ++q) project_point<T>(v0[q], v1[q], v2[q], t + Tp * q, k1, k2, g);
    reg_fft<T>(v0, g.ax[0], t, Tp, tw, true, xl + m, Mb);
    reg_fft<T>(v1, g.ax[0], t, Tp, tw, true, xl + m, Mb);
    reg_fft<T>(v2, g.ax[0], t, Tp, tw, true, xl + m, Mb);
    if (valid) {
#pragma unroll
      for (int q = 0; q < kRegP; ++q) {
        const long long e = (long long)(t + Tp * q) * S;
        base[e] = v0[q];
        base[cstride + e] = v1[q];
        base[2 * cstride + e] = v2[q];
      }
    }
    return;
  }

  const int M = sizeof(T) == 8 ? g.m64 : g.m32;
  cx<T>* bufA = tw + N0;
  cx<T>* bufB = bufA + N0 * M;
  const int nkb = (H + M - 1) / M;
  const int i = local / (N1 * nkb);
  const int rem = local - i * N1 * nkb;
  const int k1 = rem / nkb, kb = rem - k1 * nkb;
  const int Mt = min(M, H - kb * M);
  const int total = N0 * M;
  cx<T>* base0 = S0 + (long long)k1 * H + kb * M;

  cx<T> reg[3][kMaxPpt];
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    cx<T>* base = base0 + (3 * i + l) * cstride;
    for (int t = threadIdx.x; t < total; t += kThreads) {
      const int e = t / M, m = t - e * M;
      bufA[t] = m < Mt ? base[e * S + m] : cx<T>{(T)0, (T)0};
    }
    __syncthreads();
    const cx<T>* R = fft_lds<T>(bufA, bufB, g.ax[0], M, 1, M, tw, false, true);
#pragma unroll
    for (int pt = 0; pt < kMaxPpt; ++pt) {
      const int t = threadIdx.x + pt * kThreads;
      if (t < total) reg[l][pt] = R[t];
    }
    __syncthreads();
  }
#pragma unroll
  for (int pt = 0; pt < kMaxPpt; ++pt) {
    const int t = threadIdx.x + pt * kThreads;
    if (t < total) {
      const int k0 = t / M, m = t - k0 * M;
      if (m < Mt)
        project_point<T>(reg[0][pt], reg[1][pt], reg[2][pt], k0, k1, kb * M + m, g);
      else
        reg[0][pt] = reg[1][pt] = reg[2][pt] = cx<T>{(T)0, (T)0};
    }
  }
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    cx<T>* base = base0 + (3 * i + l) * cstride;
#pragma unroll
    for (int pt = 0; pt < kMaxPpt; ++pt) {
      const int t = threadIdx.x + pt * kThreads;
      if (t < total) bufA[t] = reg[l][pt];
    }
    __syncthreads();
    const cx<T>* R = fft_lds<T>(bufA, bufB, g.ax[0], M, 1, M, tw, true, true);
    for (int t = threadIdx.x; t < total; t += kThreads) {
      const int e = t / M, m = t - e * M;
      if (m < Mt) base[e * S + m] = R[t];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Pass 5: the a2 inverse (complex-to-real) transform.  The half spectra of a
// component pair are recombined as Z = X + iY over the full line using the
// Hermitian symmetry of real fields (X[-k] = conj X[k]; the k = 0 values are
// taken real; an even line's Nyquist entry is zero), transformed back, and
// Re / Im give the two real components.
// ---------------------------------------------------------------------------
template <typename T, int MODE, typename TO>
__global__ __launch_bounds__(kThreads) void k_inv_a2(Batch B, const cx<T>* __restrict__ spec, TO* __restrict__ out,
                                                     const TO* __restrict__ p, TO* __restrict__ x, double scale,
                                                     const CgState* __restrict__ cg) {
  int local;
  const int rv = find_rve(B, K_ROW, blockIdx.x, local);
  if (skip_rve(B, MODE == INV_PW ? cg : nullptr, rv)) return;
  const Grid& g = B.grids[rv];
  extern __shared__ unsigned char smem_raw[];
  const int N2 = g.n2, RT = g.rt, H = g.h;
  const int npen = 5 * RT;
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* bufA = tw + N2;
  cx<T>* bufB = bufA + npen * N2;
  load_twiddles<T>(tw, B, g.ax[2].tw, N2);

  const long long row0 = (long long)local * RT;
  const long long srow = g.rows * H;
  const cx<T>* S = spec + g.spec_off;

  if (g.ax[2].reg) {
    // register engine: pencil slot m = pair * RT + line (slots >= 5 RT idle);
    // the pair line Z = X + iY is read straight from the half spectra (mirror
    // half conjugated), transformed in registers, written straight out.
    const int Tp = N2 / kRegP;
    const int m = threadIdx.x / Tp, t = threadIdx.x - m * Tp;
    const int pq = m / RT, rl = m - pq * RT;
    const long long row = row0 + rl;
    const bool valid = m < npen && row < g.rows;
    const int c0 = pq < 4 ? 2 * pq : 8;
    cx<T> v[kRegP];
#pragma unroll
    for (int q = 0; q < kRegP; ++q) {
      const int k = t + Tp * q;
      cx<T> z = {(T)0, (T)0};
      if (valid && 2 * k != N2) {
        const bool mirror = k >= H;
        const int kk = mirror ? N2 - k : k;
        cx<T> X = S[c0 * srow + row * H + kk];
        cx<T> Y = pq < 4 ? S[(c0 + 1) * srow + row * H + kk] : cx<T>{(T)0, (T)0};
        if (k == 0) {
          X.y = (T)0;
          Y.y = (T)0;
        }
        if (mirror) {
          X.y = -X.y;
          Y.y = -Y.y;
        }
        z = cx<T>{X.x - Y.y, X.y + Y.x};
      }
      v[q] = z;
    }
    reg_fft<T>(v, g.ax[2], t, Tp, tw, true, bufA + m * N2, 1);
    double acc[1] = {0.0};
    if (valid) {
      const long long n = g.n;
      const long long base = 9 * g.vox_off + row * N2;
      const int nc = pq < 4 ? 2 : 1;
#pragma unroll
      for (int q = 0; q < kRegP; ++q) {
        const long long v0 = base + t + Tp * q;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (h >= nc) break;
          const long long idx = v0 + (c0 + h) * n;
          const T w = h == 0 ? v[q].x : v[q].y;
          if (MODE == INV_OUT) {
            const T o = (T)scale * w;
            out[idx] = (TO)o;
            acc[0] += (double)o * (double)o;
          } else if (MODE == INV_PW) {
            out[idx] = (TO)w;
            acc[0] += (double)p[idx] * (double)(TO)w;
          } else {  // INV_RHS
            const T o = (T)scale * w;
            out[idx] = (TO)o;
            x[idx] = (TO)0;
            acc[0] += (double)o * (double)o;
          }
        }
      }
    }
    double res[1];
    block_sums<1>(acc, res);
    if (threadIdx.x == 0) pslot(B, MODE == INV_PW ? SLOT_PW : SLOT_BB)[blockIdx.x] = res[0];
    return;
  }

  for (int t = threadIdx.x; t < npen * N2; t += kThreads) {
    const int pen = t / N2, k = t - pen * N2;
    const int q = pen / RT, rl = pen - q * RT;
    const long long row = row0 + rl;
    cx<T> z = {(T)0, (T)0};
    const bool nyq = (N2 % 2 == 0) && (2 * k == N2);
    if (row < g.rows && !nyq) {
      const bool mirror = k >= H;
      const int kk = mirror ? N2 - k : k;
      const int c0 = q < 4 ? 2 * q : 8;
      cx<T> X = S[c0 * srow + row * H + kk];
      cx<T> Y = q < 4 ? S[(c0 + 1) * srow + row * H + kk] : cx<T>{(T)0, (T)0};
      if (k == 0) {
        X.y = (T)0;
        Y.y = (T)0;
      }
      if (mirror) {
        X.y = -X.y;
        Y.y = -Y.y;
      }
      z = cx<T>{X.x - Y.y, X.y + Y.x};
    }
    bufA[t] = z;
  }
  __syncthreads();
  const cx<T>* Z = fft_lds<T>(bufA, bufB, g.ax[2], npen, N2, 1, tw, true, false);

  const long long n = g.n;
  const long long off = 9 * g.vox_off;
  double acc[1] = {0.0};
  for (int t = threadIdx.x; t < RT * N2; t += kThreads) {
    const int rl = t / N2, a2 = t - rl * N2;
    const long long row = row0 + rl;
    if (row >= g.rows) continue;
    const long long v = row * N2 + a2;
    T w[9];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const cx<T> z = Z[(q * RT + rl) * N2 + a2];
      w[2 * q] = z.x;
      w[2 * q + 1] = z.y;
    }
    w[8] = Z[(4 * RT + rl) * N2 + a2].x;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      const long long idx = off + c * n + v;
      if (MODE == INV_OUT) {
        const T o = (T)scale * w[c];
        out[idx] = (TO)o;
        acc[0] += (double)o * (double)o;
      } else if (MODE == INV_PW) {
        out[idx] = (TO)w[c];
        acc[0] += (double)p[idx] * (double)(TO)w[c];
      } else {  // INV_RHS
        const T o = (T)scale * w[c];
        out[idx] = (TO)o;
        x[idx] = (TO)0;
        acc[0] += (double)o * (double)o;
      }
    }
  }
  double res[1];
  block_sums<1>(acc, res);
  if (threadIdx.x == 0) pslot(B, MODE == INV_PW ? SLOT_PW : SLOT_BB)[blockIdx.x] = res[0];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T, int LAW>
static void fwd_a2_t(int mode, const Launch& L, const Material& mat, const void* in, const void* r, void* p,
                     const void* Flin, double scale, void* spec, const CgState* cg) {
  const dim3 grid(L.nblk[K_ROW]), block(kThreads);
  const size_t lds = sizeof(T) == 8 ? L.lds_row64 : L.lds_row32;
  const T* ti = static_cast<const T*>(in);
  const T* tr = static_cast<const T*>(r);
  T* tp = static_cast<T*>(p);
  const T* tf = static_cast<const T*>(Flin);
  cx<T>* sp = static_cast<cx<T>*>(spec);
  switch (mode) {
    case FWD_COPY: hipLaunchKernelGGL((k_fwd_a2<T, FWD_COPY, MODEL_SVK>), grid, block, lds, L.s, L.b, mat, ti, tr, tp, tf, scale, sp, cg); break;
    case FWD_TANGENT: hipLaunchKernelGGL((k_fwd_a2<T, FWD_TANGENT, LAW>), grid, block, lds, L.s, L.b, mat, ti, tr, tp, tf, scale, sp, cg); break;
    case FWD_TANGENT_UNI: hipLaunchKernelGGL((k_fwd_a2<T, FWD_TANGENT_UNI, LAW>), grid, block, lds, L.s, L.b, mat, ti, tr, tp, tf, scale, sp, cg); break;
    default: hipLaunchKernelGGL((k_fwd_a2<T, FWD_CG, LAW>), grid, block, lds, L.s, L.b, mat, ti, tr, tp, tf, scale, sp, cg); break;
  }
}

void launch_fwd_a2(int prec, int mode, const Launch& L, const Material& mat, const void* in_T, const void* r_T,
                   void* p_T, const void* Flin, double scale, void* spec, const CgState* cg) {
  if (prec == PREC_F64) {
    if (mat.model == MODEL_J2)
      fwd_a2_t<double, MODEL_J2>(mode, L, mat, in_T, r_T, p_T, Flin, scale, spec, cg);
    else
      fwd_a2_t<double, MODEL_SVK>(mode, L, mat, in_T, r_T, p_T, Flin, scale, spec, cg);
  } else {
    fwd_a2_t<float, MODEL_SVK>(mode, L, mat, in_T, r_T, p_T, Flin, scale, spec, cg);  // J2 runs in FP64 only
  }
}

void launch_col_a1(int prec, bool inverse, const Launch& L, void* spec, const CgState* cg) {
  const dim3 block(kThreads);
  if (prec == PREC_F64) {
    const dim3 grid(L.nblk[K_COL1_64]);
    if (inverse)
      hipLaunchKernelGGL((k_col_a1<double, true>), grid, block, L.lds_col1_64, L.s, L.b,
                         static_cast<cx<double>*>(spec), cg);
    else
      hipLaunchKernelGGL((k_col_a1<double, false>), grid, block, L.lds_col1_64, L.s, L.b,
                         static_cast<cx<double>*>(spec), cg);
  } else {
    const dim3 grid(L.nblk[K_COL1_32]);
    if (inverse)
      hipLaunchKernelGGL((k_col_a1<float, true>), grid, block, L.lds_col1_32, L.s, L.b,
                         static_cast<cx<float>*>(spec), cg);
    else
      hipLaunchKernelGGL((k_col_a1<float, false>), grid, block, L.lds_col1_32, L.s, L.b,
                         static_cast<cx<float>*>(spec), cg);
  }
}

void launch_col_a0_project(int prec, const Launch& L, void* spec, const CgState* cg) {
  const dim3 block(kThreads);
  if (prec == PREC_F64)
    hipLaunchKernelGGL((k_col_a0_project<double>), dim3(L.nblk[K_COL0_64]), block, L.lds_col0_64, L.s, L.b,
                       static_cast<cx<double>*>(spec), cg);
  else
    hipLaunchKernelGGL((k_col_a0_project<float>), dim3(L.nblk[K_COL0_32]), block, L.lds_col0_32, L.s, L.b,
                       static_cast<cx<float>*>(spec), cg);
}

template <typename T, typename TO>
static void inv_a2_t(int mode, const Launch& L, const void* spec, void* out, const void* p, void* x, double scale,
                     const CgState* cg) {
  const dim3 grid(L.nblk[K_ROW]), block(kThreads);
  const size_t lds = sizeof(T) == 8 ? L.lds_row64 : L.lds_row32;
  const cx<T>* sp = static_cast<const cx<T>*>(spec);
  TO* to = static_cast<TO*>(out);
  const TO* tp = static_cast<const TO*>(p);
  TO* tx = static_cast<TO*>(x);
  switch (mode) {
    case INV_OUT: hipLaunchKernelGGL((k_inv_a2<T, INV_OUT, TO>), grid, block, lds, L.s, L.b, sp, to, tp, tx, scale, cg); break;
    case INV_PW: hipLaunchKernelGGL((k_inv_a2<T, INV_PW, TO>), grid, block, lds, L.s, L.b, sp, to, tp, tx, scale, cg); break;
    default: hipLaunchKernelGGL((k_inv_a2<T, INV_RHS, TO>), grid, block, lds, L.s, L.b, sp, to, tp, tx, scale, cg); break;
  }
}

void launch_inv_a2(int prec, int mode, const Launch& L, const void* spec, void* out_T, int out_prec,
                   const void* p_T, void* x_T, double scale, const CgState* cg) {
  if (prec == PREC_F64) {
    if (out_prec == PREC_F64)
      inv_a2_t<double, double>(mode, L, spec, out_T, p_T, x_T, scale, cg);
    else
      inv_a2_t<double, float>(mode, L, spec, out_T, p_T, x_T, scale, cg);
  } else {
    inv_a2_t<float, float>(mode, L, spec, out_T, p_T, x_T, scale, cg);
  }
}

}  // namespace fftnk
