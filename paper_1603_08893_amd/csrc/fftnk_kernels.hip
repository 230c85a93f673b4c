// HIP kernels of libfftnk for gfx950 (CDNA4, wave64).
//
// The projected-tangent operator of the finite-strain FFT Newton-Krylov method
// (de Geus et al. 2017, Sec. 2.5-2.6): A p = G(K(F) : p), with
//   * the tangent action K(F) : p recomputed per voxel from F (Sec. 4.3),
//   * a real-to-complex 3-D DFT of the 9 components in three passes
//     (a2 rows, a1 pencils, a0 pencils),
//   * the projection G-hat applied row by row of the tensor (App. D: G-hat_ijlm =
//     delta_im g_jl, so row i of the result only needs row i of the input),
//     fused with the a0 forward and inverse transforms,
//   * the inverse a1 and a2 passes.
// All transforms are Stockham autosort mixed-radix FFTs staged through LDS;
// no vendor FFT library is used.  Block partial sums go to fixed slots and are
// reduced in a fixed order, so every result is bitwise reproducible.
#include "fftnk_internal.h"

#include <cmath>

namespace fftnk {

// ---------------------------------------------------------------------------
// complex arithmetic
// ---------------------------------------------------------------------------
template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) {
  return {a.x + b.x, a.y + b.y};
}
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) {
  return {a.x - b.x, a.y - b.y};
}
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) {
  return {a.x * s, a.y * s};
}
// a * (+i) for the inverse direction, a * (-i) for the forward one
template <typename T>
__device__ __forceinline__ cx<T> rot(cx<T> a, bool inv) {
  return inv ? cx<T>{-a.y, a.x} : cx<T>{a.y, -a.x};
}
template <typename T>
__device__ __forceinline__ cx<T> twid(const cx<T>* tw, int e, bool inv) {
  cx<T> w = tw[e];
  if (inv) w.y = -w.y;
  return w;
}

// ---------------------------------------------------------------------------
// small DFTs in registers: v[q] <- sum_r v[r] W_R^{rq}, W_R = exp(-+2 pi i / R)
// ---------------------------------------------------------------------------
template <typename T, int R>
struct SmallDft {
  // generic odd radix through the length-n twiddle table (W_R^e = W_n^{e n/R})
  __device__ __forceinline__ static void run(cx<T>* v, const cx<T>* tw, int n, bool inv) {
    cx<T> o[R];
    const int st = n / R;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      cx<T> s = v[0];
#pragma unroll
      for (int r = 1; r < R; ++r) s = s + cmul(v[r], twid(tw, ((r * q) % R) * st, inv));
      o[q] = s;
    }
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = o[q];
  }
};

template <typename T>
struct SmallDft<T, 2> {
  __device__ __forceinline__ static void run(cx<T>* v, const cx<T>*, int, bool) {
    const cx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  }
};

template <typename T>
__device__ __forceinline__ void dft4(cx<T>& v0, cx<T>& v1, cx<T>& v2, cx<T>& v3, bool inv) {
  const cx<T> s02 = v0 + v2, d02 = v0 - v2, s13 = v1 + v3, d13 = rot(v1 - v3, inv);
  v0 = s02 + s13;
  v1 = d02 + d13;
  v2 = s02 - s13;
  v3 = d02 - d13;
}

template <typename T>
struct SmallDft<T, 4> {
  __device__ __forceinline__ static void run(cx<T>* v, const cx<T>*, int, bool inv) {
    dft4(v[0], v[1], v[2], v[3], inv);
  }
};

template <typename T>
struct SmallDft<T, 8> {
  __device__ __forceinline__ static void run(cx<T>* v, const cx<T>*, int, bool inv) {
    cx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    cx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3, inv);
    dft4(o0, o1, o2, o3, inv);
    const T h = (T)0.70710678118654752440;  // 1 / sqrt(2)
    const T s = inv ? (T)1 : (T)-1;
    o1 = cmul(o1, cx<T>{h, s * h});   // W_8
    o2 = rot(o2, inv);                // W_8^2
    o3 = cmul(o3, cx<T>{-h, s * h});  // W_8^3
    v[0] = e0 + o0;
    v[4] = e0 - o0;
    v[1] = e1 + o1;
    v[5] = e1 - o1;
    v[2] = e2 + o2;
    v[6] = e2 - o2;
    v[3] = e3 + o3;
    v[7] = e3 - o3;
  }
};

// ---------------------------------------------------------------------------
// One Stockham stage on `npen` pencils of length n held in LDS.  Element e of
// pencil m lives at m*sp + e*se.  Ns is the product of the previous radices.
// Butterfly j (0 <= j < n/R) reads e = j + r n/R, applies W_{Ns R}^{k r}
// (k = j mod Ns), does an R-point DFT and writes e = (j - k) R + k + r Ns.
// pen_fast selects which index consecutive threads walk (pencils for column
// tiles, butterflies for row tiles) so LDS accesses stay contiguous.
// ---------------------------------------------------------------------------
template <typename T, int R>
__device__ void stage_reg(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst, int n, int Ns, int npen,
                          int sp, int se, const cx<T>* tw, bool inv, bool pen_fast) {
  const int nbf = n / R;
  const int total = nbf * npen;
  const int tws = n / (Ns * R);
  for (int b = threadIdx.x; b < total; b += kThreads) {
    int m, j;
    if (pen_fast) {
      j = b / npen;
      m = b - j * npen;
    } else {
      m = b / nbf;
      j = b - m * nbf;
    }
    const cx<T>* s = src + m * sp;
    cx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = s[(j + r * nbf) * se];
    const int k = j % Ns;
    if (k != 0) {
#pragma unroll
      for (int r = 1; r < R; ++r) v[r] = cmul(v[r], twid(tw, k * r * tws, inv));
    }
    SmallDft<T, R>::run(v, tw, n, inv);
    cx<T>* d = dst + m * sp;
    const int base = (j - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) d[(base + r * Ns) * se] = v[r];
  }
}

// Stage for a prime radix R > 8: one output per thread, direct sum.
// Output q of butterfly j: sum_r x[j + r n/R] W_n^{r (k n/(Ns R) + q n/R)}.
template <typename T>
__device__ void stage_generic(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst, int n, int Ns, int R,
                              int npen, int sp, int se, const cx<T>* tw, bool inv, bool pen_fast) {
  const int nbf = n / R;
  const int total = n * npen;
  const int tws = n / (Ns * R);
  for (int b = threadIdx.x; b < total; b += kThreads) {
    int m, idx;
    if (pen_fast) {
      idx = b / npen;
      m = b - idx * npen;
    } else {
      m = b / n;
      idx = b - m * n;
    }
    const int q = idx / nbf, j = idx - q * nbf;
    const int k = j % Ns;
    const int e = k * tws + q * nbf;  // < n
    const cx<T>* s = src + m * sp;
    cx<T> acc = s[j * se];
    int er = e;
    for (int r = 1; r < R; ++r) {
      acc = acc + cmul(s[(j + r * nbf) * se], twid(tw, er, inv));
      er += e;
      if (er >= n) er -= n;
    }
    dst[m * sp + ((j - k) * R + k + q * Ns) * se] = acc;
  }
}

// Full 1-D transform of npen pencils; buffers a (input) and b (scratch)
// ping-pong.  Returns the buffer holding the result.  Caller synchronises
// before (input written) and the routine synchronises after every stage.
template <typename T>
__device__ cx<T>* fft_lds(cx<T>* a, cx<T>* b, const AxisPlan& pl, int npen, int sp, int se, const cx<T>* tw,
                          bool inv, bool pen_fast) {
  int Ns = 1;
  for (int s = 0; s < pl.nstages; ++s) {
    const int R = pl.radix[s];
    switch (R) {
      case 2: stage_reg<T, 2>(a, b, pl.n, Ns, npen, sp, se, tw, inv, pen_fast); break;
      case 3: stage_reg<T, 3>(a, b, pl.n, Ns, npen, sp, se, tw, inv, pen_fast); break;
      case 4: stage_reg<T, 4>(a, b, pl.n, Ns, npen, sp, se, tw, inv, pen_fast); break;
      case 5: stage_reg<T, 5>(a, b, pl.n, Ns, npen, sp, se, tw, inv, pen_fast); break;
      case 7: stage_reg<T, 7>(a, b, pl.n, Ns, npen, sp, se, tw, inv, pen_fast); break;
      case 8: stage_reg<T, 8>(a, b, pl.n, Ns, npen, sp, se, tw, inv, pen_fast); break;
      default: stage_generic<T>(a, b, pl.n, Ns, R, npen, sp, se, tw, inv, pen_fast); break;
    }
    __syncthreads();
    cx<T>* t = a;
    a = b;
    b = t;
    Ns *= R;
  }
  return a;
}

template <typename T>
__device__ __forceinline__ void load_twiddles(cx<T>* dst, const void* tables, int off, int n) {
  const cx<T>* src = reinterpret_cast<const cx<T>*>(tables) + off;
  for (int i = threadIdx.x; i < n; i += kThreads) dst[i] = src[i];
}

// ---------------------------------------------------------------------------
// deterministic block reduction (wave shuffles, then the 4 waves in order)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

template <int K>
__device__ __forceinline__ void block_sums(double (&v)[K], double* out /* K results, thread 0 */) {
  __shared__ double red[kThreads / 64][K > 0 ? K : 1];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double s = wave_sum(v[k]);
    if (lane == 0) red[wid][k] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
      for (int w = 0; w < kThreads / 64; ++w) s += red[w][k];
      out[k] = s;
    }
  }
}

__device__ __forceinline__ double* pslot(const PassArgs& a, int slot) {
  return a.partials + (long long)slot * a.pstride + a.slot_base;
}

// ---------------------------------------------------------------------------
// St. Venant-Kirchhoff (Sec. 4.2) and its tangent action (Sec. 4.3), per voxel.
//   S = lam tr(E) I + 2 mu E, E = (F^T F - I)/2, P = F S
//   dP = p S + F [lam tr(F^T p) I + mu (F^T p + p^T F)]
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void svk_S(const T* F, T lam, T mu, T* S) {
  T C[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) C[3 * i + j] = F[i] * F[j] + F[3 + i] * F[3 + j] + F[6 + i] * F[6 + j];
  const T trE = (T)0.5 * (C[0] + C[4] + C[8] - (T)3);
#pragma unroll
  for (int c = 0; c < 9; ++c) S[c] = mu * C[c];
  S[0] += lam * trE - mu;
  S[4] += lam * trE - mu;
  S[8] += lam * trE - mu;
}

template <typename T>
__device__ __forceinline__ void mat33(const T* A, const T* B, T* C) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}

template <typename T>
__device__ __forceinline__ void svk_tangent(const T* F, const T* p, T lam, T mu, T* out) {
  T S[9];
  svk_S(F, lam, mu, S);
  T A[9];  // F^T p
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) A[3 * i + j] = F[i] * p[j] + F[3 + i] * p[3 + j] + F[6 + i] * p[6 + j];
  const T trA = A[0] + A[4] + A[8];
  T B[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) B[3 * i + j] = mu * (A[3 * i + j] + A[3 * j + i]);
  B[0] += lam * trA;
  B[4] += lam * trA;
  B[8] += lam * trA;
  T t1[9], t2[9];
  mat33(p, S, t1);
  mat33(F, B, t2);
#pragma unroll
  for (int c = 0; c < 9; ++c) out[c] = t1[c] + t2[c];
}

__device__ __forceinline__ void material_at(const Material& mat, long long v, double& lam, double& mu) {
  const int ph = mat.phase[v];
  const double* row = mat.table + 4 * ph;
  mu = mat.mu_field ? mat.mu_field[v] : row[1];
  lam = row[0] - 2.0 * mu / 3.0;
}

// ---------------------------------------------------------------------------
// Pass 1: the a2 (fastest axis) forward transform of the 9 components, fused
// with the production of the field being transformed.  Each work-group owns
// g.rt consecutive grid lines.  Component pairs (0,1) (2,3) (4,5) (6,7) are
// packed as x + i y into one complex transform (two real transforms for the
// price of one), component 8 rides alone; the half spectra are unpacked with
// X[k] = (Z[k] + conj Z[-k]) / 2 and Y[k] = (Z[k] - conj Z[-k]) / (2i).
// ---------------------------------------------------------------------------
struct Uni9 {
  double v[9];
};

template <typename T, int MODE>
__global__ __launch_bounds__(kThreads) void k_fwd_a2(PassArgs a, Material mat, const T* __restrict__ in,
                                                     const T* __restrict__ rvec, T* __restrict__ pvec,
                                                     const T* __restrict__ Flin, Uni9 uni, double scale,
                                                     cx<T>* __restrict__ spec, const CgState* __restrict__ cg) {
  if (MODE == FWD_CG && cg->done) return;
  const Grid& g = a.g;
  extern __shared__ unsigned char smem_raw[];
  const int N2 = g.n2, RT = g.rt, H = g.h;
  const int npen = 5 * RT;
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* bufA = tw + N2;
  cx<T>* bufB = bufA + npen * N2;
  load_twiddles<T>(tw, sizeof(T) == 8 ? a.tw64 : a.tw32, g.ax[2].tw, N2);

  const long long n = g.n;
  const long long off = 9 * g.vox_off;
  const long long row0 = (long long)blockIdx.x * RT;
  double beta = 0.0;
  bool first = false;
  if (MODE == FWD_CG) {
    beta = cg->beta;
    first = cg->iter == 0;
  }
  double acc[1] = {0.0};
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
          for (int c = 0; c < 9; ++c) p[c] = (T)uni.v[c];
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
        double lam, mu;
        material_at(mat, g.vox_off + v, lam, mu);
        svk_tangent<T>(F, p, (T)lam, (T)mu, d);
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
  const cx<T>* Z = fft_lds<T>(bufA, bufB, g.ax[2], npen, N2, 1, tw, false, false);

  const long long srow = g.rows * H;
  cx<T>* S = spec + g.spec_off;
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
    if (threadIdx.x == 0) pslot(a, SLOT_YY)[blockIdx.x] = res[0];
  }
}

// ---------------------------------------------------------------------------
// Pass 2 / 4: transform along a1 (forward or inverse) in place.  A work-group
// owns g.m consecutive a2 frequencies of one (component, a0) plane: every load
// and store row is g.m contiguous complex values.
// ---------------------------------------------------------------------------
template <typename T, bool INV>
__global__ __launch_bounds__(kThreads) void k_col_a1(PassArgs a, cx<T>* __restrict__ spec,
                                                     const CgState* __restrict__ cg) {
  if (cg && cg->done) return;
  const Grid& g = a.g;
  extern __shared__ unsigned char smem_raw[];
  const int N1 = g.n1, H = g.h, M = sizeof(T) == 8 ? g.m64 : g.m32;
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* bufA = tw + N1;
  cx<T>* bufB = bufA + N1 * M;
  load_twiddles<T>(tw, sizeof(T) == 8 ? a.tw64 : a.tw32, g.ax[1].tw, N1);

  const int nkb = (H + M - 1) / M;
  const int b = blockIdx.x;
  const int c = b / (g.n0 * nkb);
  const int rem = b - c * g.n0 * nkb;
  const int a0 = rem / nkb, kb = rem - a0 * nkb;
  const int Mt = min(M, H - kb * M);
  cx<T>* base = spec + g.spec_off + (long long)c * g.rows * H + (long long)a0 * N1 * H + kb * M;
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
// Pass 3: a0 forward transform, projection, a0 inverse transform.  A work-group
// owns one tensor row i (components 3i, 3i+1, 3i+2), one a1 frequency and g.m
// consecutive a2 frequencies.  G-hat (Sec. 2.5; App. C for even axes):
//   out_ij = xi_j (sum_l xi_l A_il) / |xi|^2 / n,   xi_d = k_d / N_d,
// zero at k = 0 and whenever an even axis sits at its Nyquist index.  The 1/n of
// the inverse transform is folded in here.
// ---------------------------------------------------------------------------
constexpr int kMaxPpt = 8;  // points per thread of a pass-3 tile (n0 * m <= kMaxPpt * kThreads)

__device__ __forceinline__ int signed_freq(int k, int n) { return 2 * k > n ? k - n : k; }

template <typename T>
__global__ __launch_bounds__(kThreads) void k_col_a0_project(PassArgs a, cx<T>* __restrict__ spec,
                                                             const CgState* __restrict__ cg) {
  if (cg && cg->done) return;
  const Grid& g = a.g;
  extern __shared__ unsigned char smem_raw[];
  const int N0 = g.n0, N1 = g.n1, H = g.h, M = sizeof(T) == 8 ? g.m64 : g.m32;
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* bufA = tw + N0;
  cx<T>* bufB = bufA + N0 * M;
  load_twiddles<T>(tw, sizeof(T) == 8 ? a.tw64 : a.tw32, g.ax[0].tw, N0);

  const int nkb = (H + M - 1) / M;
  const int b = blockIdx.x;
  const int i = b / (N1 * nkb);
  const int rem = b - i * N1 * nkb;
  const int k1 = rem / nkb, kb = rem - k1 * nkb;
  const int Mt = min(M, H - kb * M);
  const long long S = (long long)N1 * H;
  const int total = N0 * M;
  cx<T>* base0 = spec + g.spec_off + (long long)k1 * H + kb * M;
  const long long cstride = g.rows * H;

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
  const int f1 = signed_freq(k1, N1);
  const bool nyq1 = (N1 % 2 == 0) && (2 * k1 == N1);
  const T inv_n = (T)g.inv_n;
#pragma unroll
  for (int pt = 0; pt < kMaxPpt; ++pt) {
    const int t = threadIdx.x + pt * kThreads;
    if (t < total) {
      const int k0 = t / M, m = t - k0 * M;
      const int k2 = kb * M + m;
      const int f0 = signed_freq(k0, N0);
      const bool zero = (f0 == 0 && f1 == 0 && k2 == 0) || nyq1 || ((N0 % 2 == 0) && (2 * k0 == N0)) || m >= Mt;
      if (zero) {
#pragma unroll
        for (int l = 0; l < 3; ++l) reg[l][pt] = cx<T>{(T)0, (T)0};
      } else {
        const T xi[3] = {(T)f0 / (T)N0, (T)f1 / (T)N1, (T)k2 / (T)g.n2};
        const T xx = xi[0] * xi[0] + xi[1] * xi[1] + xi[2] * xi[2];
        cx<T> s = cscale(reg[0][pt], xi[0]);
        s = s + cscale(reg[1][pt], xi[1]);
        s = s + cscale(reg[2][pt], xi[2]);
        const T coef = inv_n / xx;
#pragma unroll
        for (int l = 0; l < 3; ++l) reg[l][pt] = cscale(s, xi[l] * coef);
      }
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
__global__ __launch_bounds__(kThreads) void k_inv_a2(PassArgs a, const cx<T>* __restrict__ spec,
                                                     TO* __restrict__ out, const TO* __restrict__ p,
                                                     TO* __restrict__ x, double scale,
                                                     const CgState* __restrict__ cg) {
  if (MODE == INV_PW && cg->done) return;
  const Grid& g = a.g;
  extern __shared__ unsigned char smem_raw[];
  const int N2 = g.n2, RT = g.rt, H = g.h;
  const int npen = 5 * RT;
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* bufA = tw + N2;
  cx<T>* bufB = bufA + npen * N2;
  load_twiddles<T>(tw, sizeof(T) == 8 ? a.tw64 : a.tw32, g.ax[2].tw, N2);

  const long long row0 = (long long)blockIdx.x * RT;
  const long long srow = g.rows * H;
  const cx<T>* S = spec + g.spec_off;
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
  if (threadIdx.x == 0) pslot(a, MODE == INV_PW ? SLOT_PW : SLOT_BB)[blockIdx.x] = res[0];
}

// ---------------------------------------------------------------------------
// CG vector updates and scalars (Sec. 2.6, Sec. 3: CG to accuracy eta_CG).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_cg_update(PassArgs a, T* __restrict__ x, T* __restrict__ r,
                                                        const T* __restrict__ p, const T* __restrict__ w,
                                                        const CgState* __restrict__ cg) {
  if (cg->done) return;
  const long long m = 9 * a.g.n;
  const long long off = 9 * a.g.vox_off;
  const T alpha = (T)cg->alpha;
  double acc[1] = {0.0};
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < m; i += (long long)gridDim.x * kThreads) {
    const T xi = x[off + i] + alpha * p[off + i];
    const T ri = r[off + i] - alpha * w[off + i];
    x[off + i] = xi;
    r[off + i] = ri;
    acc[0] += (double)ri * (double)ri;
  }
  double res[1];
  block_sums<1>(acc, res);
  if (threadIdx.x == 0) pslot(a, SLOT_RR)[blockIdx.x] = res[0];
}

// Fixed-order sum of nblk partials by one work-group.
__device__ double reduce_slot(const double* part, int nblk) {
  double s[1] = {0.0};
  for (int i = threadIdx.x; i < nblk; i += kThreads) s[0] += part[i];
  double res[1];
  block_sums<1>(s, res);
  __shared__ double bc;
  if (threadIdx.x == 0) bc = res[0];
  __syncthreads();
  return bc;
}

enum { ST_OK = 0, ST_CG_MAXIT = 5, ST_CG_BREAKDOWN = 6, ST_NONFINITE = 8 };

__global__ __launch_bounds__(kThreads) void k_cg_init(PassArgs a, int nblk, CgState* cg, double eta, int max_cg,
                                                      int stall) {
  const double bb = reduce_slot(pslot(a, SLOT_BB), nblk);
  if (threadIdx.x == 0) {
    cg->bb = bb;
    cg->rr = bb;
    cg->rr_min = bb;
    cg->stop2 = eta * eta * bb;
    cg->alpha = 0.0;
    cg->beta = 0.0;
    cg->pw = 0.0;
    cg->iter = 0;
    cg->since_min = 0;
    cg->max_cg = max_cg;
    cg->stall_limit = stall;
    cg->status = ST_OK;
    cg->done = (bb <= cg->stop2) ? 1 : 0;
  }
}

__global__ __launch_bounds__(kThreads) void k_cg_alpha(PassArgs a, int nblk, CgState* cg) {
  if (cg->done) return;
  const double pw = reduce_slot(pslot(a, SLOT_PW), nblk);
  if (threadIdx.x == 0) {
    cg->pw = pw;
    if (!(pw > 0.0) || !isfinite(pw)) {
      cg->status = ST_CG_BREAKDOWN;
      cg->done = 1;
      cg->alpha = 0.0;
    } else {
      cg->alpha = cg->rr / pw;
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_cg_beta(PassArgs a, int nblk, CgState* cg) {
  if (cg->done) return;
  const double rr = reduce_slot(pslot(a, SLOT_RR), nblk);
  if (threadIdx.x == 0) {
    cg->iter += 1;
    if (!isfinite(rr)) {
      cg->status = ST_NONFINITE;
      cg->done = 1;
    } else if (rr <= cg->stop2) {
      cg->rr = rr;
      cg->done = 1;
    } else if (cg->iter >= cg->max_cg) {
      cg->rr = rr;
      cg->status = ST_CG_MAXIT;
      cg->done = 1;
    } else {
      cg->beta = rr / cg->rr;
      cg->rr = rr;
      if (rr < cg->rr_min) {
        cg->rr_min = rr;
        cg->since_min = 0;
      } else {
        cg->since_min += 1;
      }
      if (cg->stall_limit > 0 && cg->since_min >= cg->stall_limit) cg->done = 1;  // stagnation: keep x
    }
  }
}

// ---------------------------------------------------------------------------
// Newton-level element-wise kernels (Alg. 1): F = F_t + dFbar, F += dF with the
// constitutive update, sums for the homogenised stress (voxel mean of P).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_set_F(PassArgs a, const double* __restrict__ Ft, double* __restrict__ F,
                                                    Uni9 dFbar, float* __restrict__ Flin32) {
  const long long n = a.g.n, off = 9 * a.g.vox_off;
  double acc[1] = {0.0};
  for (long long v = blockIdx.x * (long long)kThreads + threadIdx.x; v < n; v += (long long)gridDim.x * kThreads) {
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      const double ft = Ft[off + c * n + v];
      const double f = ft + dFbar.v[c];
      F[off + c * n + v] = f;
      acc[0] += f * f;
      if (Flin32) Flin32[off + c * n + v] = (float)ft;
    }
  }
  double res[1];
  block_sums<1>(acc, res);
  if (threadIdx.x == 0) pslot(a, SLOT_FF)[blockIdx.x] = res[0];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_newton_update(PassArgs a, Material mat, double* __restrict__ F,
                                                            const T* __restrict__ x, double* __restrict__ P,
                                                            float* __restrict__ Flin32) {
  const long long n = a.g.n, off = 9 * a.g.vox_off;
  double acc[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) acc[k] = 0.0;
  for (long long v = blockIdx.x * (long long)kThreads + threadIdx.x; v < n; v += (long long)gridDim.x * kThreads) {
    double f[9], S[9], Pv[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      const double d = (double)x[off + c * n + v];
      f[c] = F[off + c * n + v] + d;
      F[off + c * n + v] = f[c];
      acc[0] += d * d;
      if (Flin32) Flin32[off + c * n + v] = (float)f[c];
    }
    double lam, mu;
    material_at(mat, a.g.vox_off + v, lam, mu);
    svk_S<double>(f, lam, mu, S);
    mat33<double>(f, S, Pv);
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      P[off + c * n + v] = Pv[c];
      acc[1 + c] += Pv[c];
    }
  }
  double res[10];
  block_sums<10>(acc, res);
  if (threadIdx.x == 0) {
    pslot(a, SLOT_DF)[blockIdx.x] = res[0];
    for (int c = 0; c < 9; ++c) pslot(a, SLOT_PBAR + c)[blockIdx.x] = res[1 + c];
  }
}

__global__ __launch_bounds__(kThreads) void k_constitutive(PassArgs a, Material mat, const double* __restrict__ F,
                                                           double* __restrict__ P) {
  const long long n = a.g.n, off = 9 * a.g.vox_off;
  double acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = 0.0;
  for (long long v = blockIdx.x * (long long)kThreads + threadIdx.x; v < n; v += (long long)gridDim.x * kThreads) {
    double f[9], S[9], Pv[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) f[c] = F[off + c * n + v];
    double lam, mu;
    material_at(mat, a.g.vox_off + v, lam, mu);
    svk_S<double>(f, lam, mu, S);
    mat33<double>(f, S, Pv);
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      P[off + c * n + v] = Pv[c];
      acc[c] += Pv[c];
    }
  }
  double res[9];
  block_sums<9>(acc, res);
  if (threadIdx.x == 0)
    for (int c = 0; c < 9; ++c) pslot(a, SLOT_PBAR + c)[blockIdx.x] = res[c];
}

__global__ __launch_bounds__(kThreads) void k_field_sum(PassArgs a, const double* __restrict__ X, int slot0) {
  const long long n = a.g.n, off = 9 * a.g.vox_off;
  double acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = 0.0;
  for (long long v = blockIdx.x * (long long)kThreads + threadIdx.x; v < n; v += (long long)gridDim.x * kThreads) {
#pragma unroll
    for (int c = 0; c < 9; ++c) acc[c] += X[off + c * n + v];
  }
  double res[9];
  block_sums<9>(acc, res);
  if (threadIdx.x == 0)
    for (int c = 0; c < 9; ++c) pslot(a, slot0 + c)[blockIdx.x] = res[c];
}

// out[s] = sum of the nblk partials of slot slot0 + s; one work-group per slot.
__global__ __launch_bounds__(kThreads) void k_reduce(PassArgs a, int slot0, int nblk, double* out) {
  const double s = reduce_slot(pslot(a, slot0 + blockIdx.x), nblk);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

template <typename TI, typename TO>
__global__ __launch_bounds__(kThreads) void k_convert(const TI* __restrict__ in, TO* __restrict__ out, long long m) {
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < m; i += (long long)gridDim.x * kThreads)
    out[i] = (TO)in[i];
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_fill_zero(T* __restrict__ x, long long m) {
  for (long long i = blockIdx.x * (long long)kThreads + threadIdx.x; i < m; i += (long long)gridDim.x * kThreads)
    x[i] = (T)0;
}

// Adjoint gradient per voxel at the converged F with adjoint field w:
//   dL/dmu = (1/n) (g - w) : F . 2 dev(E),  dL/dK = (1/n) (g - w) : tr(E) F
// (S = (K - 2mu/3) tr(E) I + 2 mu E).  Accumulates (+=) so that several load
// cases on one modulus field add up.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_adjoint_grad(PassArgs a, const double* __restrict__ F,
                                                           const T* __restrict__ w, Uni9 g,
                                                           double* __restrict__ dmu, double* __restrict__ dK,
                                                           long long out_off) {
  const long long n = a.g.n, off = 9 * a.g.vox_off;
  for (long long v = blockIdx.x * (long long)kThreads + threadIdx.x; v < n; v += (long long)gridDim.x * kThreads) {
    double f[9], d[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      f[c] = F[off + c * n + v];
      d[c] = g.v[c] - (double)w[off + c * n + v];
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
    dmu[out_off + v] += smu * a.g.inv_n;
    if (dK) dK[out_off + v] += sK * trE * a.g.inv_n;
  }
}

// F = I on every voxel of one RVE (the stress-free start of Algorithm 1).
__global__ __launch_bounds__(kThreads) void k_set_identity(PassArgs a, double* __restrict__ F) {
  const long long n = a.g.n, off = 9 * a.g.vox_off;
  for (long long v = blockIdx.x * (long long)kThreads + threadIdx.x; v < n; v += (long long)gridDim.x * kThreads)
#pragma unroll
    for (int c = 0; c < 9; ++c) F[off + c * n + v] = (c % 4 == 0) ? 1.0 : 0.0;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static int elem_blocks(long long m) {
  long long b = (m + kThreads - 1) / kThreads;
  if (b > kRedBlocks) b = kRedBlocks;
  if (b < 1) b = 1;
  return (int)b;
}

int fwd_a2_blocks(const Grid& g) { return (int)((g.rows + g.rt - 1) / g.rt); }
int inv_a2_blocks(const Grid& g) { return fwd_a2_blocks(g); }

static size_t row_lds(const Grid& g, size_t csz) { return csz * ((size_t)g.n2 + 2 * 5 * (size_t)g.rt * g.n2); }
static int gm(const Grid& g, size_t csz) { return csz == 16 ? g.m64 : g.m32; }
static size_t col_lds(int nax, const Grid& g, size_t csz) { return csz * ((size_t)nax + 2 * (size_t)nax * gm(g, csz)); }

template <typename T>
static void fwd_a2_t(int mode, const PassArgs& a, const Material& mat, const void* in, const void* r, void* p,
                     const void* Flin, const double* uni, double scale, void* spec, const CgState* cg,
                     hipStream_t s) {
  Uni9 u{};
  if (uni)
    for (int c = 0; c < 9; ++c) u.v[c] = uni[c];
  const dim3 grid(fwd_a2_blocks(a.g)), block(kThreads);
  const size_t lds = row_lds(a.g, sizeof(cx<T>));
  const T* ti = static_cast<const T*>(in);
  const T* tr = static_cast<const T*>(r);
  T* tp = static_cast<T*>(p);
  const T* tf = static_cast<const T*>(Flin);
  cx<T>* sp = static_cast<cx<T>*>(spec);
  switch (mode) {
    case FWD_COPY: hipLaunchKernelGGL((k_fwd_a2<T, FWD_COPY>), grid, block, lds, s, a, mat, ti, tr, tp, tf, u, scale, sp, cg); break;
    case FWD_TANGENT: hipLaunchKernelGGL((k_fwd_a2<T, FWD_TANGENT>), grid, block, lds, s, a, mat, ti, tr, tp, tf, u, scale, sp, cg); break;
    case FWD_TANGENT_UNI: hipLaunchKernelGGL((k_fwd_a2<T, FWD_TANGENT_UNI>), grid, block, lds, s, a, mat, ti, tr, tp, tf, u, scale, sp, cg); break;
    default: hipLaunchKernelGGL((k_fwd_a2<T, FWD_CG>), grid, block, lds, s, a, mat, ti, tr, tp, tf, u, scale, sp, cg); break;
  }
}

void launch_fwd_a2(int prec, int mode, const PassArgs& a, const Material& mat, const void* in_T, const void* r_T,
                   void* p_T, const void* Flin, const double* uni, double scale, void* spec, const CgState* cg,
                   hipStream_t s) {
  if (prec == PREC_F64)
    fwd_a2_t<double>(mode, a, mat, in_T, r_T, p_T, Flin, uni, scale, spec, cg, s);
  else
    fwd_a2_t<float>(mode, a, mat, in_T, r_T, p_T, Flin, uni, scale, spec, cg, s);
}

void launch_col_a1(int prec, bool inverse, const PassArgs& a, void* spec, const CgState* cg, hipStream_t s) {
  const Grid& g = a.g;
  const int M = prec == PREC_F64 ? g.m64 : g.m32;
  const int nkb = (g.h + M - 1) / M;
  const dim3 grid(9 * g.n0 * nkb), block(kThreads);
  if (prec == PREC_F64) {
    const size_t lds = col_lds(g.n1, g, sizeof(cx<double>));
    if (inverse)
      hipLaunchKernelGGL((k_col_a1<double, true>), grid, block, lds, s, a, static_cast<cx<double>*>(spec), cg);
    else
      hipLaunchKernelGGL((k_col_a1<double, false>), grid, block, lds, s, a, static_cast<cx<double>*>(spec), cg);
  } else {
    const size_t lds = col_lds(g.n1, g, sizeof(cx<float>));
    if (inverse)
      hipLaunchKernelGGL((k_col_a1<float, true>), grid, block, lds, s, a, static_cast<cx<float>*>(spec), cg);
    else
      hipLaunchKernelGGL((k_col_a1<float, false>), grid, block, lds, s, a, static_cast<cx<float>*>(spec), cg);
  }
}

void launch_col_a0_project(int prec, const PassArgs& a, void* spec, const CgState* cg, hipStream_t s) {
  const Grid& g = a.g;
  const int M = prec == PREC_F64 ? g.m64 : g.m32;
  const int nkb = (g.h + M - 1) / M;
  const dim3 grid(3 * g.n1 * nkb), block(kThreads);
  if (prec == PREC_F64)
    hipLaunchKernelGGL((k_col_a0_project<double>), grid, block, col_lds(g.n0, g, sizeof(cx<double>)), s, a,
                       static_cast<cx<double>*>(spec), cg);
  else
    hipLaunchKernelGGL((k_col_a0_project<float>), grid, block, col_lds(g.n0, g, sizeof(cx<float>)), s, a,
                       static_cast<cx<float>*>(spec), cg);
}

template <typename T, typename TO>
static void inv_a2_t(int mode, const PassArgs& a, const void* spec, void* out, const void* p, void* x, double scale,
                     const CgState* cg, hipStream_t s) {
  const dim3 grid(inv_a2_blocks(a.g)), block(kThreads);
  const size_t lds = row_lds(a.g, sizeof(cx<T>));
  const cx<T>* sp = static_cast<const cx<T>*>(spec);
  TO* to = static_cast<TO*>(out);
  const TO* tp = static_cast<const TO*>(p);
  TO* tx = static_cast<TO*>(x);
  switch (mode) {
    case INV_OUT: hipLaunchKernelGGL((k_inv_a2<T, INV_OUT, TO>), grid, block, lds, s, a, sp, to, tp, tx, scale, cg); break;
    case INV_PW: hipLaunchKernelGGL((k_inv_a2<T, INV_PW, TO>), grid, block, lds, s, a, sp, to, tp, tx, scale, cg); break;
    default: hipLaunchKernelGGL((k_inv_a2<T, INV_RHS, TO>), grid, block, lds, s, a, sp, to, tp, tx, scale, cg); break;
  }
}

void launch_inv_a2(int prec, int mode, const PassArgs& a, const void* spec, void* out_T, int out_prec,
                   const void* p_T, void* x_T, double scale, const CgState* cg, hipStream_t s) {
  if (prec == PREC_F64) {
    if (out_prec == PREC_F64)
      inv_a2_t<double, double>(mode, a, spec, out_T, p_T, x_T, scale, cg, s);
    else
      inv_a2_t<double, float>(mode, a, spec, out_T, p_T, x_T, scale, cg, s);
  } else {
    inv_a2_t<float, float>(mode, a, spec, out_T, p_T, x_T, scale, cg, s);
  }
}

void launch_cg_update(int prec, const PassArgs& a, void* x, void* r, const void* p, const void* w, CgState* cg,
                      hipStream_t s) {
  const int nb = elem_blocks(9 * a.g.n);
  if (prec == PREC_F64)
    hipLaunchKernelGGL((k_cg_update<double>), dim3(nb), dim3(kThreads), 0, s, a, static_cast<double*>(x),
                       static_cast<double*>(r), static_cast<const double*>(p), static_cast<const double*>(w), cg);
  else
    hipLaunchKernelGGL((k_cg_update<float>), dim3(nb), dim3(kThreads), 0, s, a, static_cast<float*>(x),
                       static_cast<float*>(r), static_cast<const float*>(p), static_cast<const float*>(w), cg);
}

void launch_cg_alpha(const PassArgs& a, int nblk_pw, CgState* cg, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(kThreads), 0, s, a, nblk_pw, cg);
}

void launch_cg_beta(const PassArgs& a, CgState* cg, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(kThreads), 0, s, a, elem_blocks(9 * a.g.n), cg);
}

void launch_cg_init(const PassArgs& a, int nblk_bb, CgState* cg, double eta, int max_cg, int stall, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(kThreads), 0, s, a, nblk_bb, cg, eta, max_cg, stall);
}

int elem_blocks_vox(const Grid& g) { return elem_blocks(g.n); }

void launch_set_F(const PassArgs& a, const double* Ft, double* F, const double* dFbar, float* Flin32, hipStream_t s) {
  Uni9 u{};
  for (int c = 0; c < 9; ++c) u.v[c] = dFbar[c];
  hipLaunchKernelGGL(k_set_F, dim3(elem_blocks(a.g.n)), dim3(kThreads), 0, s, a, Ft, F, u, Flin32);
}

void launch_newton_update(int prec, const PassArgs& a, const Material& mat, double* F, const void* x, double* P,
                          float* Flin32, hipStream_t s) {
  const int nb = elem_blocks(a.g.n);
  if (prec == PREC_F64)
    hipLaunchKernelGGL((k_newton_update<double>), dim3(nb), dim3(kThreads), 0, s, a, mat, F,
                       static_cast<const double*>(x), P, Flin32);
  else
    hipLaunchKernelGGL((k_newton_update<float>), dim3(nb), dim3(kThreads), 0, s, a, mat, F,
                       static_cast<const float*>(x), P, Flin32);
}

void launch_constitutive(const PassArgs& a, const Material& mat, const double* F, double* P, hipStream_t s) {
  hipLaunchKernelGGL(k_constitutive, dim3(elem_blocks(a.g.n)), dim3(kThreads), 0, s, a, mat, F, P);
}

void launch_field_sum(const PassArgs& a, const double* X, int slot0, hipStream_t s) {
  hipLaunchKernelGGL(k_field_sum, dim3(elem_blocks(a.g.n)), dim3(kThreads), 0, s, a, X, slot0);
}

void launch_reduce(const PassArgs& a, int slot0, int nslots, int nblk, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(nslots), dim3(kThreads), 0, s, a, slot0, nblk, out);
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

void launch_adjoint_grad(int prec, const PassArgs& a, const double* F, const void* w, const double* g, double* dmu,
                         double* dK, long long out_off, hipStream_t s) {
  Uni9 u{};
  for (int c = 0; c < 9; ++c) u.v[c] = g[c];
  const int nb = elem_blocks(a.g.n);
  if (prec == PREC_F64)
    hipLaunchKernelGGL((k_adjoint_grad<double>), dim3(nb), dim3(kThreads), 0, s, a, F, static_cast<const double*>(w),
                       u, dmu, dK, out_off);
  else
    hipLaunchKernelGGL((k_adjoint_grad<float>), dim3(nb), dim3(kThreads), 0, s, a, F, static_cast<const float*>(w),
                       u, dmu, dK, out_off);
}

void launch_set_identity(const PassArgs& a, double* F, hipStream_t s) {
  hipLaunchKernelGGL(k_set_identity, dim3(elem_blocks(a.g.n)), dim3(kThreads), 0, s, a, F);
}

void launch_fill_zero(int prec, void* x, long long count, hipStream_t s) {
  const int nb = elem_blocks(count);
  if (prec == PREC_F64)
    hipLaunchKernelGGL((k_fill_zero<double>), dim3(nb), dim3(kThreads), 0, s, static_cast<double*>(x), count);
  else
    hipLaunchKernelGGL((k_fill_zero<float>), dim3(nb), dim3(kThreads), 0, s, static_cast<float*>(x), count);
}

}  // namespace fftnk
