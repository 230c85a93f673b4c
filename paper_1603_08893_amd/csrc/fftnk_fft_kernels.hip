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
int row1_blocks(const Grid& g) { return (int)((g.rows + g.rt1 - 1) / g.rt1); }

// pencils per work-group of the register engine (P = the axis plan's points per thread)
static int reg_pencils(const AxisPlan& pl) { return kThreads / (pl.n / pl.reg); }

int col1_blocks(const Grid& g, int prec) {
  if (g.ax[1].reg) {
    long long np = 9LL * g.n0 * g.h, mb = reg_pencils(g.ax[1]);
    if (prec == PREC_F32 && col_engine(g.ax[1].reg, g.n1, g.h, g.spec_off, 4) == 16) mb *= 2;
    return (int)((np + mb - 1) / mb);
  }
  const int M = prec == PREC_F64 ? g.m64 : g.m32;
  return (int)((9LL * g.n0 * g.h + M - 1) / M);
}

int col0_blocks(const Grid& g, int prec) {
  if (g.ax[0].reg) {
    long long np = 3LL * g.n1 * g.h, mb = reg_pencils(g.ax[0]);
    if (prec == PREC_F32 && col_engine(g.ax[0].reg, g.n0, g.h, g.spec_off, 4) == 16) mb *= 2;
    return (int)((np + mb - 1) / mb);
  }
  const int M = prec == PREC_F64 ? g.m64 : g.m32;
  return 3 * (int)(((long long)g.n1 * g.h + M - 1) / M);
}

// ---------------------------------------------------------------------------
// Pass 1: a2 forward transform of the 9 components, fused with the production
// of the field being transformed.  Each work-group owns g.rt1 consecutive grid
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
    if (mat.j2t) {  // the compact tangent stored for this linearisation point
      double t[kJ2Tan];
#pragma unroll
      for (int k = 0; k < kJ2Tan; ++k) t[k] = __builtin_nontemporal_load(mat.j2t + k * mat.ntot + gv);
      j2_tangent_compact(F, h, t, p, d);
    } else {
      j2_tangent(F, h, K, mu, ty0, H, p, d);
    }
  } else {
    double lam, mu;
    material_at(mat, gv, lam, mu);
    svk_tangent<T>(F, p, (T)lam, (T)mu, d);
  }
}

// Identity choice at Nyquist frequencies (App. C) on an even a2 axis: the a2
// Nyquist plane is not stored, and G-hat = identity there makes its round trip
// through passes 2-4 return every line's own coefficient times n0 n1 / n.  So
// pass 1 keeps z = Z[n2 / 2] of a pencil (real parts: the coefficients of the
// pair's two components, both real) divided by n2, and pass 5 puts it back.
template <typename T, typename G>
__device__ __forceinline__ void put_nyquist(const Batch& B, const G& g, long long row, int pq, cx<T> z) {
  T* ny = static_cast<T*>(B.nyq) + 9 * g.row_off + row;
  const T s = (T)1 / (T)g.n2;
  if (pq == 4) {
    ny[8 * g.rows] = s * z.x;
  } else {
    ny[(2 * pq) * g.rows] = s * z.x;
    ny[(2 * pq + 1) * g.rows] = s * z.y;
  }
}
template <typename T, typename G>
__device__ __forceinline__ cx<T> get_nyquist(const Batch& B, const G& g, long long row, int pq) {
  const T* ny = static_cast<const T*>(B.nyq) + 9 * g.row_off + row;
  if (pq == 4) return cx<T>{ny[8 * g.rows], (T)0};
  return cx<T>{ny[(2 * pq) * g.rows], ny[(2 * pq + 1) * g.rows]};
}

// store of one half-spectrum entry by pass 1 (non-temporal in CG mode when
// the policy says so)
template <int MODE, typename T>
__device__ __forceinline__ void st_spec(cx<T>* p, cx<T> v) {
  if constexpr (MODE == FWD_CG && (nt_policy<T>() & NT_P1_STORE_SPEC) != 0) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    __builtin_nontemporal_store(v2{v.x, v.y}, reinterpret_cast<v2*>(p));
  } else {
    *p = v;
  }
}

template <typename T, int MODE, int LAW, int ENG, bool NTOP>
__device__ __forceinline__ void tile_fwd_a2(const Batch& B, const Material& mat, const T* __restrict__ in,
                                            const T* __restrict__ rvec, T* __restrict__ pvec, T* __restrict__ xvec,
                                            const T* __restrict__ Flin, double scale, cx<T>* __restrict__ spec,
                                            const CgState* __restrict__ cg, const int b) {
  int local;
  const int rv = find_rve(B, K_ROW1, b, local);
  if (skip_rve(B, MODE == FWD_CG ? cg : nullptr, rv)) return;
  const auto& g = grid_of(B, rv);
  if (pass1_engine(g.ax[2].reg) != ENG) return;  // another engine's launch owns this cell
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const int N2 = g.n2, RT = g.rt1, H = g.h;
  const int npen = 5 * RT;
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* bufA = tw + padded_len(N2);
  cx<T>* bufB = bufA + npen * N2;
  load_twiddles<T>(tw, B, g.ax[2].tw, N2);

  const long long n = g.n;
  const long long off = 9 * g.vox_off;
  const long long row0 = (long long)local * RT;
  // partial sum: <p, K p> (FWD_CG) or ||K p||^2 / ||field||^2 (the projected field's norm)
  double acc[1] = {0.0};
  // register engine: pencil slot m = pair * RT + line (slots >= 5 RT idle),
  // stage the field in LDS once, transform in registers, unpack through one
  // mirror exchange.  bufA holds one slot of padded_len(N2) entries per pencil.
  constexpr bool reg = ENG != 0;
  const int SL = reg ? padded_len(N2) : N2;  // LDS slot of one line
  if ((int)threadIdx.x < RT * N2) {  // rt1 * n2 <= kThreads: at most one voxel per thread
    const int t = threadIdx.x;
    const int rl = t / N2, a2 = t - rl * N2;
    const long long row = row0 + rl;
    T d[9];
    if (row < g.rows) {
      const long long v = row * N2 + a2;
      // uniform component base + 32-bit byte offset of the voxel (n <= 512^2 256 = 2^26);
      // every load below is issued before any arithmetic uses it
      const unsigned vb = (unsigned)v * (unsigned)sizeof(T);
      if (MODE == FWD_COPY) {
#pragma unroll
        for (int c = 0; c < 9; ++c) d[c] = (T)scale * *byte_off(in + off + c * n, vb);
#pragma unroll
        for (int c = 0; c < 9; ++c) acc[0] += (double)d[c] * (double)d[c];
      } else {
        T p[9], F[9];
        if (MODE == FWD_TANGENT_UNI) {
#pragma unroll
          for (int c = 0; c < 9; ++c) p[c] = (T)cptr(B.uni)[9 * rv + c];
#pragma unroll
          for (int c = 0; c < 9; ++c) F[c] = *byte_off(Flin + off + c * n, vb);
        } else if (MODE == FWD_TANGENT) {
#pragma unroll
          for (int c = 0; c < 9; ++c) p[c] = ld_stream_if<NTOP, NT_OP_LOAD_P>(byte_off(in + off + c * n, vb));
#pragma unroll
          for (int c = 0; c < 9; ++c) F[c] = *byte_off(Flin + off + c * n, vb);
        } else {  // FWD_CG, iteration k: p_k goes to slot k mod W
          const int k = cptr(cg)[rv].iter, W = B.xwin;
          T* pnew = pvec + (long long)(k % W) * B.vstride;
          if (k == 0) {  // p_0 = r_0, x_0 = 0
#pragma unroll
            for (int c = 0; c < 9; ++c) p[c] = ld_stream<NT_P1_LOAD_VEC>(byte_off(rvec + off + c * n, vb));
#pragma unroll
            for (int c = 0; c < 9; ++c) F[c] = ld_stream<NT_P1_LOAD_F>(byte_off(Flin + off + c * n, vb));
          } else {  // p_k = r + beta p_{k-1}
            const T beta = (T)cptr(cg)[rv].beta;
            const T* pold = pvec + (long long)((k - 1) % W) * B.vstride;
            T po[9];
#pragma unroll
            for (int c = 0; c < 9; ++c) {
              p[c] = ld_stream<NT_P1_LOAD_VEC>(byte_off(rvec + off + c * n, vb));
              po[c] = ld_stream<NT_P1_LOAD_VEC>(byte_off(pold + off + c * n, vb));
            }
#pragma unroll
            for (int c = 0; c < 9; ++c) F[c] = ld_stream<NT_P1_LOAD_F>(byte_off(Flin + off + c * n, vb));
            if (k % W == 0) {
              // start of a window: slots 0 .. W-1 hold p_{k-W} .. p_{k-1} (the last
              // one is p_old); x += alpha_j p_j in the order of j, as the updates of
              // the single iterations would (the same roundings)
              T xo[9];
#pragma unroll
              for (int c = 0; c < 9; ++c) xo[c] = ld_stream<NT_P1_LOAD_VEC>(byte_off(xvec + off + c * n, vb));
#pragma unroll 1
              for (int i = 0; i < W - 1; ++i) {
                const T a = (T)cptr(cg)[rv].ahist[i];
                const T* pi = pvec + (long long)i * B.vstride;
                T q[9];
#pragma unroll
                for (int c = 0; c < 9; ++c) q[c] = ld_stream<NT_P1_LOAD_VEC>(byte_off(pi + off + c * n, vb));
#pragma unroll
                for (int c = 0; c < 9; ++c) xo[c] = xo[c] + a * q[c];
              }
              const T a = (T)cptr(cg)[rv].ahist[W - 1];
#pragma unroll
              for (int c = 0; c < 9; ++c) st_stream<NT_P1_STORE_VEC>(byte_off(xvec + off + c * n, vb), xo[c] + a * po[c]);
            }
#pragma unroll
            for (int c = 0; c < 9; ++c) p[c] = p[c] + beta * po[c];
          }
#pragma unroll
          for (int c = 0; c < 9; ++c) st_stream<NT_P1_STORE_VEC>(byte_off(pnew + off + c * n, vb), p[c]);
        }
        tangent_at<T, LAW>(mat, g.vox_off + v, F, p, d);
        if (MODE == FWD_CG) {
#pragma unroll
          for (int c = 0; c < 9; ++c) acc[0] += (double)p[c] * (double)d[c];
        } else {
#pragma unroll
          for (int c = 0; c < 9; ++c) acc[0] += (double)d[c] * (double)d[c];
        }
      }
    } else {
#pragma unroll
      for (int c = 0; c < 9; ++c) d[c] = (T)0;
    }
    const int ea = reg ? lpad(a2) : a2;
#pragma unroll
    for (int q = 0; q < 4; ++q) bufA[(q * RT + rl) * SL + ea] = cx<T>{d[2 * q], d[2 * q + 1]};
    bufA[(4 * RT + rl) * SL + ea] = cx<T>{d[8], (T)0};
  }
  __syncthreads();
  const long long srow = g.rows * H;
  cx<T>* S = spec + g.spec_off;

  if constexpr (ENG != 0) {
    constexpr int P = ENG;  // points per thread of the register engine
    const int Tp = N2 / P;
    const int m = threadIdx.x / Tp, t = threadIdx.x - m * Tp;
    // idle pencil slots (m >= 5 rt1) all work in one spare slot after the
    // used ones: their values are never read back into anything stored
    cx<T>* xl = bufA + min(m, npen) * SL;
    cx<T> v[P];
#pragma unroll
    for (int q = 0; q < P; ++q) v[q] = xl[lpad(t + Tp * q)];
    __syncthreads();
    reg_fft<T, true, P>(v, N2, t, tw, false, xl);
#pragma unroll
    for (int q = 0; q < P; ++q) xl[lpad(t + Tp * q)] = v[q];
    __syncthreads();
    const int pq = m / RT, rl = m - pq * RT;
    const long long row = row0 + rl;
    if (m < npen && row < g.rows) {
#pragma unroll
      for (int q = 0; q < P / 2; ++q) {  // k = t + Tp q < n2 / 2 = h
        const int k = t + Tp * q;
        const cx<T> z = v[q];
        const cx<T> zm = xl[lpad(k ? N2 - k : 0)];
        if (pq == 4) {
          st_spec<MODE>(S + 8 * srow + row * H + k, z);
        } else {
          st_spec<MODE>(S + (2 * pq) * srow + row * H + k, cx<T>{(T)0.5 * (z.x + zm.x), (T)0.5 * (z.y - zm.y)});
          st_spec<MODE>(S + (2 * pq + 1) * srow + row * H + k, cx<T>{(T)0.5 * (z.y + zm.y), (T)-0.5 * (z.x - zm.x)});
        }
      }
      // lane 0 holds k = n2 / 2 at q = P / 2: the two real Nyquist coefficients
      if (g.nyq_id && t == 0) put_nyquist<T>(B, g, row, pq, v[P / 2]);
    }
    double res[1];
    block_sums<1>(acc, res);
    if (threadIdx.x == 0) pslot(B, MODE == FWD_CG ? SLOT_PW : SLOT_YY)[b] = res[0];
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
  if (g.nyq_id && (N2 & 1) == 0) {
    for (int t = threadIdx.x; t < npen; t += kThreads) {
      const int pq = t / RT, rl = t - pq * RT;
      const long long row = row0 + rl;
      if (row < g.rows) put_nyquist<T>(B, g, row, pq, Z[t * N2 + N2 / 2]);
    }
  }
  double res[1];
  block_sums<1>(acc, res);
  if (threadIdx.x == 0) pslot(B, MODE == FWD_CG ? SLOT_PW : SLOT_YY)[b] = res[0];
}

template <typename T, int MODE, int LAW, int ENG, bool NTOP = true>
__global__ __launch_bounds__(kThreads) void k_fwd_a2(Batch B, Material mat, const T* __restrict__ in,
                                                     const T* __restrict__ rvec, T* __restrict__ pvec,
                                                     T* __restrict__ xvec, const T* __restrict__ Flin, double scale,
                                                     cx<T>* __restrict__ spec, const CgState* __restrict__ cg) {
  // tiles in reverse order: pass 1 starts on the grid lines that the previous
  // pass 5 wrote last (still in the last-level cache); see k_col_a0_project
  tile_fwd_a2<T, MODE, LAW, ENG, NTOP>(B, mat, in, rvec, pvec, xvec, Flin, scale, spec, cg, gridDim.x - 1 - blockIdx.x);
}

// ---------------------------------------------------------------------------
// Pass 2 / 4: transform along a1 (forward or inverse) in place.
// Register engine: kThreads / (n1/8) pencils per work-group, consecutive in
// (component, a0, k2) order so that each load / store row of the work-group is
// a run of consecutive k2.  LDS engine: g.m pencils consecutive in the same
// order (several planes where a plane has fewer k2).
// ---------------------------------------------------------------------------
template <typename T, bool INV, int ENG>
__device__ __forceinline__ void tile_col_a1(const Batch& B, cx<T>* __restrict__ spec, const CgState* cg,
                                            const int b) {
  int local;
  const int rv = find_rve(B, sizeof(T) == 8 ? K_COL1_64 : K_COL1_32, b, local);
  if (skip_rve(B, cg, rv)) return;
  const auto& g = grid_of(B, rv);
  if (col_engine(g.ax[1].reg, g.n1, g.h, g.spec_off, sizeof(T)) != ENG) return;  // another launch owns this cell
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const int N1 = g.n1, H = g.h;
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  load_twiddles<T>(tw, B, g.ax[1].tw, N1);
  cx<T>* S0 = spec + g.spec_off;

  if constexpr (ENG != 0) {
    constexpr int P = ENG == 16 ? 8 : ENG;  // points per thread of the register engine
    cx<T>* xl = tw + padded_len(N1);
    const int Tp = N1 / P, Mb = kThreads / Tp;
    const int m = threadIdx.x % Mb, t = threadIdx.x / Mb;
    const long long npen = 9LL * g.n0 * H;
    if constexpr (ENG == 16) {
      // pencils pen, pen + 1 (same k2 line): one 16-byte access per element
      long long pen = 2 * ((long long)local * Mb + m);
      const bool valid = pen < npen;  // npen is even here
      if (!valid) pen = 0;
      const long long plane = pen / H;
      cx2<T>* base = reinterpret_cast<cx2<T>*>(S0 + plane * N1 * H + (pen - plane * H));
      const long long hs = H / 2;  // a row of the spectrum in pairs
      cx<T> va[P], vb[P];
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const cx2<T> w = valid ? base[(long long)(t + Tp * q) * hs] : cx2<T>{};
        va[q] = w.a;
        vb[q] = w.b;
      }
      reg_fft<T, false, P>(va, N1, t, tw, INV, xl + m);
      reg_fft<T, false, P>(vb, N1, t, tw, INV, xl + m);
      if (valid) {
#pragma unroll
        for (int q = 0; q < P; ++q) base[(long long)(t + Tp * q) * hs] = cx2<T>{va[q], vb[q]};
      }
      return;
    }
    long long pen = (long long)local * Mb + m;
    const bool valid = pen < npen;
    if (!valid) pen = 0;
    const long long plane = pen / H;
    cx<T>* base = S0 + plane * N1 * H + (pen - plane * H);
    cx<T> v[P];
#pragma unroll
    for (int q = 0; q < P; ++q) v[q] = valid ? base[(long long)(t + Tp * q) * H] : cx<T>{(T)0, (T)0};
    reg_fft<T, false, P>(v, N1, t, tw, INV, xl + m);
    if (valid) {
#pragma unroll
      for (int q = 0; q < P; ++q) base[(long long)(t + Tp * q) * H] = v[q];
    }
    return;
  }

  // M consecutive pencils of the (component, a0, k2) order: pencil
  // P = plane H + k2 holds its element e at plane N1 H + e H + k2.  Loads and
  // stores give consecutive lanes consecutive k2 (m fastest), or, where a
  // plane holds fewer than 64 bytes of k2, consecutive elements of one pencil.
  const int M = sizeof(T) == 8 ? g.m64 : g.m32;
  cx<T>* bufA = tw + padded_len(N1);
  cx<T>* bufB = bufA + N1 * M;
  const int npen = 9 * g.n0 * H;
  const int P0 = local * M;
  const int Mt = min(M, npen - P0);
  const bool efast = H * (int)sizeof(cx<T>) < 64;
  auto at = [&](int e, int m) {
    const int P = P0 + m, plane = P / H, k2 = P - plane * H;
    return S0 + (long long)plane * N1 * H + (long long)e * H + k2;
  };
  for (int t = threadIdx.x; t < N1 * M; t += kThreads) {
    const int m = efast ? t / N1 : t % M, e = efast ? t - m * N1 : t / M;
    bufA[e * M + m] = m < Mt ? *at(e, m) : cx<T>{(T)0, (T)0};
  }
  __syncthreads();
  const cx<T>* R = fft_lds<T>(bufA, bufB, g.ax[1], M, 1, M, tw, INV, true);
  for (int t = threadIdx.x; t < N1 * M; t += kThreads) {
    const int m = efast ? t / N1 : t % M, e = efast ? t - m * N1 : t / M;
    if (m < Mt) *at(e, m) = R[e * M + m];
  }
}

template <typename T, bool INV, int ENG>
__global__ __launch_bounds__(kThreads) void k_col_a1(Batch B, cx<T>* __restrict__ spec, const CgState* cg,
                                                     CgState* alpha_cg) {
  // the first nrve work-groups of a CG iteration's forward launch compute the
  // step lengths from the first pass's partial sums (alpha_cg == cg); a
  // breakdown found there marks its RVE done while this launch runs, which
  // may skip part of that RVE's tiles: harmless, its CG is over
  const int na = alpha_cg ? B.nrve : 0;
  if ((int)blockIdx.x < na) {
    cg_alpha_group(B, alpha_cg, blockIdx.x);
    return;
  }
  tile_col_a1<T, INV, ENG>(B, spec, cg, (int)blockIdx.x - na);
}

// ---------------------------------------------------------------------------
// Pass 3: a0 forward transform, projection, a0 inverse transform.  A pencil is
// one (tensor row i, k1, k2) triple carrying the three components 3i..3i+2:
// G-hat_ijlm = delta_im g_jl (App. D), so row i of the projected field needs
// row i of the input only.  G-hat (Sec. 2.5; App. C for even axes):
//   out_ij = xi_j (sum_l xi_l A_il) / |xi|^2 / n,   xi_d = k_d / N_d,
// zero at k = 0 and whenever an even axis sits at its Nyquist index (or, with
// the identity choice of App. C, the identity there).  The 1/n of the inverse
// transform is folded in here.
// ---------------------------------------------------------------------------

// One frequency of the projection with the identity choice at Nyquist
// frequencies (the a2 index of the stored half spectrum is never Nyquist).
template <typename T, typename G>
__device__ __forceinline__ void project_point(cx<T>& a0, cx<T>& a1, cx<T>& a2, int k0, int k1, int k2,
                                              const G& g, T rn0, T rn1, T rn2 /* 1 / N_d */) {
  const int f0 = signed_freq(k0, g.n0), f1 = signed_freq(k1, g.n1);
  if (f0 == 0 && f1 == 0 && k2 == 0) {
    a0 = a1 = a2 = cx<T>{(T)0, (T)0};
    return;
  }
  if (((g.n0 % 2 == 0) && (2 * k0 == g.n0)) || ((g.n1 % 2 == 0) && (2 * k1 == g.n1))) {
    const T s = (T)g.inv_n;
    a0 = cscale(a0, s);
    a1 = cscale(a1, s);
    a2 = cscale(a2, s);
    return;
  }
  const T xi0 = (T)f0 * rn0, xi1 = (T)f1 * rn1, xi2 = (T)k2 * rn2;
  const T coef = (T)g.inv_n / (xi0 * xi0 + xi1 * xi1 + xi2 * xi2);
  cx<T> s = cscale(a0, xi0);
  s = s + cscale(a1, xi1);
  s = s + cscale(a2, xi2);
  a0 = cscale(s, xi0 * coef);
  a1 = cscale(s, xi1 * coef);
  a2 = cscale(s, xi2 * coef);
}

// One pencil (tensor row i, k1, k2) of pass 3 on the register engine, held as
// v[component][point]: transform, project, transform back, in place.  Two
// forward and two inverse transforms (the scheme of the single-pencil path of
// tile_col_a0_project), or three of each with the identity choice at Nyquist
// frequencies (ID).
template <typename T, int P, bool ID, typename G>
__device__ __forceinline__ void reg_pencil_project(cx<T> (&v)[3][P], const G& g, int k1, int k2, int t,
                                                   const cx<T>* tw, cx<T>* xl, T rn0, T rn1, T rn2) {
  const int N0 = g.n0, Tp = N0 / P;
  if constexpr (ID) {
#pragma unroll
    for (int c = 0; c < 3; ++c) reg_fft<T, false, P>(v[c], N0, t, tw, false, xl);
#pragma unroll
    for (int q = 0; q < P; ++q) project_point(v[0][q], v[1][q], v[2][q], t + Tp * q, k1, k2, g, rn0, rn1, rn2);
#pragma unroll
    for (int c = 0; c < 3; ++c) reg_fft<T, false, P>(v[c], N0, t, tw, true, xl);
  } else {
    const int f1 = signed_freq(k1, g.n1);
    const T xi1 = (T)f1 * rn1, xi2 = (T)k2 * rn2;
    const bool pen_zero = (g.n1 % 2 == 0) && (2 * k1 == g.n1);
#pragma unroll
    for (int q = 0; q < P; ++q) v[1][q] = cscale(v[1][q], xi1) + cscale(v[2][q], xi2);
    reg_fft<T, false, P>(v[1], N0, t, tw, false, xl);
    reg_fft<T, false, P>(v[0], N0, t, tw, false, xl);
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const int k0 = t + Tp * q;
      const int f0 = signed_freq(k0, N0);
      const T xi0 = (T)f0 * rn0;
      const bool zero = pen_zero || (f0 == 0 && f1 == 0 && k2 == 0) || ((N0 % 2 == 0) && (2 * k0 == N0));
      const T c = zero ? (T)0 : (T)g.inv_n / (xi0 * xi0 + xi1 * xi1 + xi2 * xi2);
      const cx<T> sc = cscale(cscale(v[0][q], xi0) + v[1][q], c);
      v[0][q] = cscale(sc, xi0);
      v[1][q] = sc;
    }
    reg_fft<T, false, P>(v[0], N0, t, tw, true, xl);
    reg_fft<T, false, P>(v[1], N0, t, tw, true, xl);
#pragma unroll
    for (int q = 0; q < P; ++q) {
      v[2][q] = cscale(v[1][q], xi2);
      v[1][q] = cscale(v[1][q], xi1);
    }
  }
}

// Pass 3 on the register engine for FP32 pencils taken in k2-adjacent pairs
// (col_engine 16): every load and store is one 16-byte access covering both
// pencils of the pair, each pencil transformed and projected on its own.
template <typename T, int P, bool ID, typename G>
__device__ __forceinline__ void col_a0_project_pairs(const G& g, cx<T>* __restrict__ S0, const cx<T>* tw, cx<T>* xl,
                                                     int local, int Mb, int m, int t, T rn0, T rn1, T rn2) {
  const int N0 = g.n0, N1 = g.n1, H = g.h;
  const int Tp = N0 / P;
  const long long S2 = (long long)N1 * H / 2;  // element stride along a0, in pairs
  const long long cstride2 = g.rows * H / 2;
  const long long npen = 3LL * N1 * H;
  long long pen = 2 * ((long long)local * Mb + m);
  const bool valid = pen < npen;  // npen is even here
  if (!valid) pen = 0;
  const long long qq = pen / H;
  const int k2 = (int)(pen - qq * H);
  const int i = (int)(qq / N1), k1 = (int)(qq - (long long)i * N1);
  cx2<T>* base = reinterpret_cast<cx2<T>*>(S0) + (long long)(3 * i) * cstride2 + ((long long)k1 * H + k2) / 2 +
                 (long long)t * S2;
  auto at = [&](int c, int q) { return base + (long long)c * cstride2 + (long long)q * Tp * S2; };
  cx<T> va[3][P], vb[3][P];  // the two pencils of the pair, [component][point]
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const cx2<T> v = valid ? *at(c, q) : cx2<T>{};
      va[c][q] = v.a;
      vb[c][q] = v.b;
    }
  reg_pencil_project<T, P, ID>(va, g, k1, k2, t, tw, xl, rn0, rn1, rn2);
  reg_pencil_project<T, P, ID>(vb, g, k1, k2 + 1, t, tw, xl, rn0, rn1, rn2);
  if (valid) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int q = 0; q < P; ++q) *at(c, q) = cx2<T>{va[c][q], vb[c][q]};
  }
}

template <typename T, int ENG>
__device__ __forceinline__ void tile_col_a0_project(const Batch& B, cx<T>* __restrict__ spec,
                                                             const CgState* __restrict__ cg, const int b) {
  int local;
  const int rv = find_rve(B, sizeof(T) == 8 ? K_COL0_64 : K_COL0_32, b, local);
  if (skip_rve(B, cg, rv)) return;
  const auto& g = grid_of(B, rv);
  if (col_engine(g.ax[0].reg, g.n0, g.h, g.spec_off, sizeof(T)) != ENG) return;  // another launch owns this cell
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const int N0 = g.n0, N1 = g.n1, H = g.h;
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  load_twiddles<T>(tw, B, g.ax[0].tw, N0);
  cx<T>* S0 = spec + g.spec_off;
  const long long S = (long long)N1 * H;  // element stride along a0
  const long long cstride = g.rows * H;
  const T rn0 = (T)1 / (T)N0, rn1 = (T)1 / (T)N1, rn2 = (T)1 / (T)g.n2;

  if constexpr (ENG != 0) {
    constexpr int P = ENG == 16 ? 8 : ENG;  // points per thread of the register engine
    cx<T>* xl = tw + padded_len(N0);
    const int Tp = N0 / P, Mb = kThreads / Tp;
    const int m = threadIdx.x % Mb, t = threadIdx.x / Mb;
    const long long npen = 3LL * N1 * H;
    if constexpr (ENG == 16) {
      col_a0_project_pairs<T, P, false>(g, S0, tw, xl + m, local, Mb, m, t, rn0, rn1, rn2);
      return;
    }
    long long pen = (long long)local * Mb + m;
    const bool valid = pen < npen;
    if (!valid) pen = 0;
    const long long qq = pen / H;
    const int k2 = (int)(pen - qq * H);
    const int i = (int)(qq / N1), k1 = (int)(qq - (long long)i * N1);
    // byte offset of the lane's first element inside the cell's spectrum (32
    // bits: at most 9 n0 n1 h entries); the per-(component, q) parts are
    // uniform, so loads and stores use a scalar base plus this one register
    const unsigned lo =
        (unsigned)(((long long)(3 * i) * cstride + (long long)k1 * H + k2 + (long long)t * S) * (long long)sizeof(cx<T>));
    char* sb = reinterpret_cast<char*>(S0);
    auto at = [&](int c, int q) {
      return reinterpret_cast<cx<T>*>(sb + ((long long)c * cstride + (long long)q * Tp * S) * (long long)sizeof(cx<T>) + lo);
    };
    // Along the pencil k1, k2 are fixed, so xi_1, xi_2 are constants and the
    // a0 transform commutes with them: with s = sum_l xi_l A_il,
    //   s = xi_0 FFT(a_i0) + FFT(xi_1 a_i1 + xi_2 a_i2),
    //   out_i0 = IFFT(xi_0 c s),  out_i1 = xi_1 IFFT(c s),  out_i2 = xi_2 IFFT(c s),
    // c = (1/n) / |xi|^2 (zero at k = 0 and at an even axis' Nyquist index):
    // two forward and two inverse transforms instead of three of each.
    const int f1 = signed_freq(k1, N1);
    const T xi1 = (T)f1 * rn1, xi2 = (T)k2 * rn2;
    const bool pen_zero = (N1 % 2 == 0) && (2 * k1 == N1);
    cx<T> v0[P], v1[P];
    {
      cx<T> v2[P];
#pragma unroll
      for (int q = 0; q < P; ++q) {
        v0[q] = valid ? *at(0, q) : cx<T>{(T)0, (T)0};
        v1[q] = valid ? *at(1, q) : cx<T>{(T)0, (T)0};
        v2[q] = valid ? *at(2, q) : cx<T>{(T)0, (T)0};
      }
#pragma unroll
      for (int q = 0; q < P; ++q) v1[q] = cscale(v1[q], xi1) + cscale(v2[q], xi2);
    }
    reg_fft<T, false, P>(v1, N0, t, tw, false, xl + m);
    reg_fft<T, false, P>(v0, N0, t, tw, false, xl + m);
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const int k0 = t + Tp * q;
      const int f0 = signed_freq(k0, N0);
      const T xi0 = (T)f0 * rn0;
      const bool zero = pen_zero || (f0 == 0 && f1 == 0 && k2 == 0) || ((N0 % 2 == 0) && (2 * k0 == N0));
      const T c = zero ? (T)0 : (T)g.inv_n / (xi0 * xi0 + xi1 * xi1 + xi2 * xi2);
      const cx<T> sc = cscale(cscale(v0[q], xi0) + v1[q], c);
      v0[q] = cscale(sc, xi0);
      v1[q] = sc;
    }
    reg_fft<T, false, P>(v0, N0, t, tw, true, xl + m);
    reg_fft<T, false, P>(v1, N0, t, tw, true, xl + m);
    if (valid) {
#pragma unroll
      for (int q = 0; q < P; ++q) {
        *at(0, q) = v0[q];
        *at(1, q) = cscale(v1[q], xi1);
        *at(2, q) = cscale(v1[q], xi2);
      }
    }
    return;
  }

  // M consecutive pencils P = k1 H + k2 of one tensor row: in every a0 plane
  // of the row's components they sit at offsets P, one run of M entries
  const int M = sizeof(T) == 8 ? g.m64 : g.m32;
  cx<T>* bufA = tw + padded_len(N0);
  cx<T>* bufB = bufA + N0 * M;
  const int npen = N1 * H;
  const int ntile = (npen + M - 1) / M;
  const int i = local / ntile;
  const int P0 = (local - i * ntile) * M;
  const int Mt = min(M, npen - P0);
  const int total = N0 * M;

  // The same two-forward / two-inverse scheme as the register engine, with
  // xi_1, xi_2 per pencil.  Every load is issued before the first transform.
  cx<T>* b0 = S0 + (long long)(3 * i) * cstride + P0;
  cx<T> ra[kMaxPpt], ru[kMaxPpt];  // a_i0, then FFT(a_i0); u = xi1 a_i1 + xi2 a_i2, then FFT(u)
#pragma unroll
  for (int pt = 0; pt < kMaxPpt; ++pt) {
    const int t = threadIdx.x + pt * kThreads;
    const int e = t / M, m = t - e * M;
    const bool ok = t < total && m < Mt;
    const long long o = ok ? (long long)e * S + m : 0;
    const cx<T> a0 = b0[o], a1 = b0[cstride + o], a2 = b0[2 * cstride + o];
    const int k1 = (P0 + m) / H, k2 = P0 + m - k1 * H;
    const T xi1 = (T)signed_freq(k1, N1) * rn1, xi2 = (T)k2 * rn2;
    ra[pt] = ok ? a0 : cx<T>{(T)0, (T)0};
    ru[pt] = ok ? cscale(a1, xi1) + cscale(a2, xi2) : cx<T>{(T)0, (T)0};
  }
#pragma unroll
  for (int l = 0; l < 2; ++l) {  // forward: u, then a_i0
    cx<T>(&r)[kMaxPpt] = l == 0 ? ru : ra;
#pragma unroll
    for (int pt = 0; pt < kMaxPpt; ++pt) {
      const int t = threadIdx.x + pt * kThreads;
      if (t < total) bufA[t] = r[pt];
    }
    __syncthreads();
    const cx<T>* Rz = fft_lds<T>(bufA, bufB, g.ax[0], M, 1, M, tw, false, true);
#pragma unroll
    for (int pt = 0; pt < kMaxPpt; ++pt) {
      const int t = threadIdx.x + pt * kThreads;
      if (t < total) r[pt] = Rz[t];
    }
    __syncthreads();
  }
  // s = xi0 A0 + U; ra <- xi0 c s, ru <- c s, c = (1/n) / |xi|^2 (0 on k = 0 and Nyquist)
#pragma unroll
  for (int pt = 0; pt < kMaxPpt; ++pt) {
    const int t = threadIdx.x + pt * kThreads;
    const int k0 = t / M, m = t - k0 * M;
    const int k1 = (P0 + m) / H, k2 = P0 + m - k1 * H;
    const int f0 = signed_freq(k0, N0), f1 = signed_freq(k1, N1);
    const T xi0 = (T)f0 * rn0, xi1 = (T)f1 * rn1, xi2 = (T)k2 * rn2;
    const bool pen_zero = (N1 % 2 == 0) && (2 * k1 == N1);
    const bool zero = pen_zero || m >= Mt || (f0 == 0 && f1 == 0 && k2 == 0) || ((N0 % 2 == 0) && (2 * k0 == N0));
    const T c = zero ? (T)0 : (T)g.inv_n / (xi0 * xi0 + xi1 * xi1 + xi2 * xi2);
    const cx<T> sc = cscale(cscale(ra[pt], xi0) + ru[pt], c);
    ra[pt] = cscale(sc, xi0);
    ru[pt] = sc;
  }
#pragma unroll
  for (int l = 0; l < 2; ++l) {  // inverse: xi0 c s -> component 0; c s -> components 1 and 2
    cx<T>(&r)[kMaxPpt] = l == 0 ? ra : ru;
#pragma unroll
    for (int pt = 0; pt < kMaxPpt; ++pt) {
      const int t = threadIdx.x + pt * kThreads;
      if (t < total) bufA[t] = r[pt];
    }
    __syncthreads();
    const cx<T>* Rz = fft_lds<T>(bufA, bufB, g.ax[0], M, 1, M, tw, true, true);
    for (int t = threadIdx.x; t < total; t += kThreads) {
      const int e = t / M, m = t - e * M;
      if (m >= Mt) continue;
      const long long o = (long long)e * S + m;
      if (l == 0) {
        b0[o] = Rz[t];
      } else {
        const int k1 = (P0 + m) / H, k2 = P0 + m - k1 * H;
        const T xi1 = (T)signed_freq(k1, N1) * rn1, xi2 = (T)k2 * rn2;
        b0[cstride + o] = cscale(Rz[t], xi1);
        b0[2 * cstride + o] = cscale(Rz[t], xi2);
      }
    }
    __syncthreads();
  }
}

// Pass 3 with the identity choice at Nyquist frequencies (App. C): there the
// three components of a row are kept apart, so the two-transform shortcut
// above does not apply; three forward transforms, the projection point by
// point, three inverse transforms.  Same tiles as the default variant.
template <typename T, int ENG>
__device__ __forceinline__ void tile_col_a0_project_id(const Batch& B, cx<T>* __restrict__ spec,
                                                       const CgState* __restrict__ cg, const int b) {
  int local;
  const int rv = find_rve(B, sizeof(T) == 8 ? K_COL0_64 : K_COL0_32, b, local);
  if (skip_rve(B, cg, rv)) return;
  const auto& g = grid_of(B, rv);
  if (col_engine(g.ax[0].reg, g.n0, g.h, g.spec_off, sizeof(T)) != ENG) return;  // another launch owns this cell
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const int N0 = g.n0, N1 = g.n1, H = g.h;
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  load_twiddles<T>(tw, B, g.ax[0].tw, N0);
  cx<T>* S0 = spec + g.spec_off;
  const long long S = (long long)N1 * H;  // element stride along a0
  const long long cstride = g.rows * H;
  const T rn0 = (T)1 / (T)N0, rn1 = (T)1 / (T)N1, rn2 = (T)1 / (T)g.n2;

  if constexpr (ENG != 0) {
    constexpr int P = ENG == 16 ? 8 : ENG;
    cx<T>* xl = tw + padded_len(N0);
    const int Tp = N0 / P, Mb = kThreads / Tp;
    const int m = threadIdx.x % Mb, t = threadIdx.x / Mb;
    const long long npen = 3LL * N1 * H;
    if constexpr (ENG == 16) {
      col_a0_project_pairs<T, P, true>(g, S0, tw, xl + m, local, Mb, m, t, rn0, rn1, rn2);
      return;
    }
    long long pen = (long long)local * Mb + m;
    const bool valid = pen < npen;
    if (!valid) pen = 0;
    const long long qq = pen / H;
    const int k2 = (int)(pen - qq * H);
    const int i = (int)(qq / N1), k1 = (int)(qq - (long long)i * N1);
    cx<T>* p0 = S0 + (long long)(3 * i) * cstride + (long long)k1 * H + k2 + (long long)t * S;
    cx<T> v[3][P];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int q = 0; q < P; ++q) v[c][q] = valid ? p0[c * cstride + (long long)q * Tp * S] : cx<T>{(T)0, (T)0};
#pragma unroll
    for (int c = 0; c < 3; ++c) reg_fft<T, false, P>(v[c], N0, t, tw, false, xl + m);
#pragma unroll
    for (int q = 0; q < P; ++q) project_point(v[0][q], v[1][q], v[2][q], t + Tp * q, k1, k2, g, rn0, rn1, rn2);
#pragma unroll
    for (int c = 0; c < 3; ++c) reg_fft<T, false, P>(v[c], N0, t, tw, true, xl + m);
    if (valid) {
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int q = 0; q < P; ++q) p0[c * cstride + (long long)q * Tp * S] = v[c][q];
    }
    return;
  }

  const int M = sizeof(T) == 8 ? g.m64 : g.m32;
  cx<T>* bufA = tw + padded_len(N0);
  cx<T>* bufB = bufA + N0 * M;
  const int npen = N1 * H;
  const int ntile = (npen + M - 1) / M;
  const int i = local / ntile;
  const int P0 = (local - i * ntile) * M;
  const int Mt = min(M, npen - P0);
  const int total = N0 * M;
  cx<T>* b0 = S0 + (long long)(3 * i) * cstride + P0;
  cx<T> r[3][kMaxPpt];
#pragma unroll
  for (int pt = 0; pt < kMaxPpt; ++pt) {
    const int t = threadIdx.x + pt * kThreads;
    const int e = t / M, m = t - e * M;
    const bool ok = t < total && m < Mt;
    const long long o = ok ? (long long)e * S + m : 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) r[c][pt] = ok ? b0[c * cstride + o] : cx<T>{(T)0, (T)0};
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int pt = 0; pt < kMaxPpt; ++pt) {
      const int t = threadIdx.x + pt * kThreads;
      if (t < total) bufA[t] = r[c][pt];
    }
    __syncthreads();
    const cx<T>* Rz = fft_lds<T>(bufA, bufB, g.ax[0], M, 1, M, tw, false, true);
#pragma unroll
    for (int pt = 0; pt < kMaxPpt; ++pt) {
      const int t = threadIdx.x + pt * kThreads;
      if (t < total) r[c][pt] = Rz[t];
    }
    __syncthreads();
  }
#pragma unroll
  for (int pt = 0; pt < kMaxPpt; ++pt) {
    const int t = threadIdx.x + pt * kThreads;
    const int k0 = t / M, m = t - k0 * M;
    const int k1 = (P0 + m) / H, k2 = P0 + m - k1 * H;
    if (t < total && m < Mt) project_point(r[0][pt], r[1][pt], r[2][pt], k0, k1, k2, g, rn0, rn1, rn2);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int pt = 0; pt < kMaxPpt; ++pt) {
      const int t = threadIdx.x + pt * kThreads;
      if (t < total) bufA[t] = r[c][pt];
    }
    __syncthreads();
    const cx<T>* Rz = fft_lds<T>(bufA, bufB, g.ax[0], M, 1, M, tw, true, true);
    for (int t = threadIdx.x; t < total; t += kThreads) {
      const int e = t / M, m = t - e * M;
      if (m < Mt) b0[c * cstride + (long long)e * S + m] = Rz[t];
    }
    __syncthreads();
  }
}

// Three work-groups per CU, but two (256 VGPRs) where the registers of a
// pencil's transforms do not fit otherwise: FP64 12-point pencils, the
// identity choice's three transforms and FP32 pencil pairs under it; one
// (accumulation registers too) for the identity choice's three FP64 12-point
// transforms.
template <typename T, int ENG, bool NYQ_ID>
constexpr int a0_groups_per_cu() {
  if (ENG == 16) return NYQ_ID ? 2 : 3;
  if (sizeof(T) == 8 && NYQ_ID && ENG == 12) return 1;
  return (sizeof(T) == 8 && (ENG == 12 || (NYQ_ID && ENG != 0))) || (NYQ_ID && ENG == 12) ? 2 : 3;
}

template <typename T, int ENG, bool NYQ_ID>
__global__ __launch_bounds__(kThreads, (a0_groups_per_cu<T, ENG, NYQ_ID>())) void k_col_a0_project(
    Batch B, cx<T>* __restrict__ spec, const CgState* __restrict__ cg) {
  // Consecutive passes alternate their direction through memory (pass 1
  // reversed, 2 forward, 3 reversed, 4 and 5 forward) so that each starts on
  // what the previous one touched last: 2-4 % per CG iteration at 128^3 and
  // 192^3, where the fields exceed the 256 MB last-level cache in part or whole.
  const int b = gridDim.x - 1 - blockIdx.x;
  if constexpr (NYQ_ID)
    tile_col_a0_project_id<T, ENG>(B, spec, cg, b);
  else
    tile_col_a0_project<T, ENG>(B, spec, cg, b);
}

// ---------------------------------------------------------------------------
// Pass 5: the a2 inverse (complex-to-real) transform.  The half spectra of a
// component pair are recombined as Z = X + iY over the full line using the
// Hermitian symmetry of real fields (X[-k] = conj X[k]; the k = 0 values are
// taken real; an even line's Nyquist entry is zero, or what pass 1 kept for
// the identity choice at Nyquist frequencies), transformed back, and
// Re / Im give the two real components.
// ---------------------------------------------------------------------------
template <typename T, int MODE, typename TO, int ENG, bool NTOP>
__device__ __forceinline__ void tile_inv_a2(const Batch& B, const cx<T>* __restrict__ spec, TO* __restrict__ out,
                                            TO* __restrict__ x, double scale,
                                                     const CgState* __restrict__ cg, const int b) {
  int local;
  const int rv = find_rve(B, K_ROW, b, local);
  if (skip_rve(B, MODE == INV_CGR ? cg : nullptr, rv)) return;
  const auto& g = grid_of(B, rv);
  if (g.ax[2].reg != ENG) return;  // another engine's launch owns this cell
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  const int N2 = g.n2, RT = g.rt, H = g.h;
  const int npen = 5 * RT;
  cx<T>* tw = reinterpret_cast<cx<T>*>(smem_raw);
  cx<T>* bufA = tw + padded_len(N2);
  cx<T>* bufB = bufA + npen * N2;
  load_twiddles<T>(tw, B, g.ax[2].tw, N2);

  const long long row0 = (long long)local * RT;
  const long long srow = g.rows * H;
  const cx<T>* S = spec + g.spec_off;

  if constexpr (ENG != 0) {
    constexpr int P = ENG;  // points per thread of the register engine
    // register engine: pencil slot m = pair * RT + line (slots >= 5 RT idle);
    // the pair line Z = X + iY is read straight from the half spectra (mirror
    // half conjugated), transformed in registers, written straight out.
    const int Tp = N2 / P;
    const int m = threadIdx.x / Tp, t = threadIdx.x - m * Tp;
    const int pq = m / RT, rl = m - pq * RT;
    const long long row = row0 + rl;
    const bool valid = m < npen && row < g.rows;
    const int c0 = pq < 4 ? 2 * pq : 8;
    // Thread t loads the stored half line at k = t + Tp q, q < P / 2 (all
    // of k < h = n2 / 2, each entry once, addresses clamped into the cell).
    // The upper half k = n2 - k' needs conj X[k'], held by lane (Tp - t) mod Tp
    // of the same pencil at q' = P - 1 - q (lane 0 holds its own at
    // q' = P - q; q = P / 2 is the Nyquist index: zero, or with the identity
    // choice the coefficient pass 1 kept).
    constexpr int P2 = P / 2;
    const cx<T>* SX = S + c0 * srow + (valid ? row : row0) * H;
    const cx<T>* SY = pq < 4 ? SX + srow : SX;
    cx<T> X[P2], Y[P2];
#pragma unroll
    for (int q = 0; q < P2; ++q) {
      X[q] = SX[t + Tp * q];
      Y[q] = SY[t + Tp * q];
    }
    const T yon = pq < 4 ? (T)1 : (T)0;  // component 8 rides alone
    cx<T> v[P];
#pragma unroll
    for (int q = 0; q < P2; ++q) {
      const T xi = (t == 0 && q == 0) ? (T)0 : X[q].y;  // k = 0 taken real
      const T yi = (t == 0 && q == 0) ? (T)0 : yon * Y[q].y;
      v[q] = valid ? cx<T>{X[q].x - yi, xi + yon * Y[q].x} : cx<T>{(T)0, (T)0};
    }
    const int src = (Tp - t) & (Tp - 1);
    // lane 0's Nyquist entry: zero, or the kept coefficients (identity choice)
    cx<T> zn = {(T)0, (T)0};
    if (g.nyq_id && t == 0 && valid) zn = get_nyquist<T>(B, g, row, pq);
#pragma unroll
    for (int q = P2; q < P; ++q) {
      cx<T> xm, ym;
      xm.x = __shfl(X[P - 1 - q].x, src, Tp);
      xm.y = __shfl(X[P - 1 - q].y, src, Tp);
      ym.x = __shfl(Y[P - 1 - q].x, src, Tp);
      ym.y = __shfl(Y[P - 1 - q].y, src, Tp);
      if (t == 0) {
        xm = q == P2 ? cx<T>{zn.x, (T)0} : X[q == P2 ? 0 : P - q];
        ym = q == P2 ? cx<T>{zn.y, (T)0} : Y[q == P2 ? 0 : P - q];
      }
      const T xi = -xm.y, yi = -yon * ym.y;  // conjugated
      v[q] = valid ? cx<T>{xm.x - yi, xi + yon * ym.x} : cx<T>{(T)0, (T)0};
    }
    reg_fft<T, true, P>(v, N2, t, tw, true, bufA + min(m, npen) * padded_len(N2));  // idle slots share a spare one
    double acc[1] = {0.0};
    if (valid) {
      const long long n = g.n;
      const long long base = 9 * g.vox_off + row * N2;
      const int nc = pq < 4 ? 2 : 1;
      const T alpha = MODE == INV_CGR ? (T)cptr(cg)[rv].alpha : (T)0;
      TO rin[P][2];  // INV_CGR: the residual, all loads issued before use
      if (MODE == INV_CGR) {
#pragma unroll
        for (int q = 0; q < P; ++q)
#pragma unroll
          for (int h = 0; h < 2; ++h)
            rin[q][h] = h < nc ? ld_stream<NT_P5_LOAD_R>(out + base + t + Tp * q + (c0 + h) * n) : (TO)0;
      }
#pragma unroll
      for (int q = 0; q < P; ++q) {
        const long long v0 = base + t + Tp * q;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (h >= nc) break;
          const long long idx = v0 + (c0 + h) * n;
          const T w = h == 0 ? v[q].x : v[q].y;
          if (MODE == INV_OUT) {
            const T o = (T)scale * w;
            st_stream_if<NTOP, NT_OP_STORE_OUT>(out + idx, (TO)o);
            acc[0] += (double)o * (double)o;
          } else if (MODE == INV_CGR) {
            const TO rn = (TO)((T)rin[q][h] - alpha * w);
            st_stream<NT_P5_STORE_R>(out + idx, rn);
            acc[0] += (double)rn * (double)rn;
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
    if (threadIdx.x == 0) pslot(B, MODE == INV_CGR ? SLOT_RR : SLOT_BB)[b] = res[0];
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
    } else if (row < g.rows && g.nyq_id) {
      z = get_nyquist<T>(B, g, row, q);
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
    TO rin[9];  // INV_CGR: the residual, all loads issued before use
    if (MODE == INV_CGR) {
#pragma unroll
      for (int c = 0; c < 9; ++c) rin[c] = out[off + c * n + v];
    }
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      const long long idx = off + c * n + v;
      if (MODE == INV_OUT) {
        const T o = (T)scale * w[c];
        out[idx] = (TO)o;
        acc[0] += (double)o * (double)o;
      } else if (MODE == INV_CGR) {
        const TO rn = (TO)((T)rin[c] - (T)cptr(cg)[rv].alpha * w[c]);
        out[idx] = rn;
        acc[0] += (double)rn * (double)rn;
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
  if (threadIdx.x == 0) pslot(B, MODE == INV_CGR ? SLOT_RR : SLOT_BB)[b] = res[0];
}

template <typename T, int MODE, typename TO, int ENG, bool NTOP = true>
__global__ __launch_bounds__(kThreads) void k_inv_a2(Batch B, const cx<T>* __restrict__ spec, TO* __restrict__ out,
                                                     TO* __restrict__ x, double scale,
                                                     const CgState* __restrict__ cg) {
  tile_inv_a2<T, MODE, TO, ENG, NTOP>(B, spec, out, x, scale, cg, blockIdx.x);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// One work-group per tile: the hardware dispatcher staggers the work-groups'
// load, transform and store phases better than a resident tile loop does
// (measured on the 128^3 operator).
template <typename... KArgs, typename... Args>
static void launch_tiles(void (*kernel)(KArgs...), int ntiles, size_t lds, hipStream_t s, Args... args) {
  if (ntiles < 1) return;
  hipLaunchKernelGGL(kernel, dim3(ntiles), dim3(kThreads), lds, s, args...);
}

// Each pass has a register-engine and an LDS-engine kernel (separate, so that
// neither carries the other's register budget); a launch starts the variants
// the batch needs (Launch::eng, per axis: bit 0 some cell on the LDS engine,
// bit 1 on the 8-point register engine, bit 2 on the 12-point one) and each
// skips the others' cells.
template <typename T, int MODE, int LAW, bool NTOP = true>
static void fwd_a2_mode(const Launch& L, const Material& mat, const T* in, const T* r, T* p, T* x, const T* Flin,
                        double scale, cx<T>* spec, const CgState* cg) {
  const int ntiles = L.nblk[K_ROW1];
  const size_t lds = sizeof(T) == 8 ? L.lds_row1_64 : L.lds_row1_32;
  // pass 1 runs 12-point axes on the LDS engine (pass1_engine)
  if (L.eng[2] & 2)
    launch_tiles(&k_fwd_a2<T, MODE, LAW, 8, NTOP>, ntiles, lds, L.s, L.b, mat, in, r, p, x, Flin, scale, spec, cg);
  if (L.eng[2] & 5)
    launch_tiles(&k_fwd_a2<T, MODE, LAW, 0, NTOP>, ntiles, lds, L.s, L.b, mat, in, r, p, x, Flin, scale, spec, cg);
}

template <typename T, int LAW>
static void fwd_a2_t(int mode, const Launch& L, const Material& mat, const void* in, const void* r, void* p,
                     void* x, const void* Flin, double scale, void* spec, const CgState* cg) {
  const T* ti = static_cast<const T*>(in);
  const T* tr = static_cast<const T*>(r);
  T* tp = static_cast<T*>(p);
  T* tx = static_cast<T*>(x);
  const T* tf = static_cast<const T*>(Flin);
  cx<T>* sp = static_cast<cx<T>*>(spec);
  switch (mode) {
    case FWD_COPY: fwd_a2_mode<T, FWD_COPY, MODEL_SVK>(L, mat, ti, tr, tp, tx, tf, scale, sp, cg); break;
    case FWD_TANGENT:
      if (L.ntop)
        fwd_a2_mode<T, FWD_TANGENT, LAW, true>(L, mat, ti, tr, tp, tx, tf, scale, sp, cg);
      else
        fwd_a2_mode<T, FWD_TANGENT, LAW, false>(L, mat, ti, tr, tp, tx, tf, scale, sp, cg);
      break;
    case FWD_TANGENT_UNI: fwd_a2_mode<T, FWD_TANGENT_UNI, LAW>(L, mat, ti, tr, tp, tx, tf, scale, sp, cg); break;
    default: fwd_a2_mode<T, FWD_CG, LAW>(L, mat, ti, tr, tp, tx, tf, scale, sp, cg); break;
  }
}

void launch_fwd_a2(int prec, int mode, const Launch& L, const Material& mat, const void* in_T, const void* r_T,
                   void* p_T, void* x_T, const void* Flin, double scale, void* spec, const CgState* cg) {
  if (prec == PREC_F64) {
    if (mat.model == MODEL_J2)
      fwd_a2_t<double, MODEL_J2>(mode, L, mat, in_T, r_T, p_T, x_T, Flin, scale, spec, cg);
    else
      fwd_a2_t<double, MODEL_SVK>(mode, L, mat, in_T, r_T, p_T, x_T, Flin, scale, spec, cg);
  } else {
    fwd_a2_t<float, MODEL_SVK>(mode, L, mat, in_T, r_T, p_T, x_T, Flin, scale, spec, cg);  // J2 runs in FP64 only
  }
}

template <typename T, bool INV>
static void col_a1_t(const Launch& L, void* spec, const CgState* cg, CgState* alpha_cg) {
  const int ntiles = L.nblk[sizeof(T) == 8 ? K_COL1_64 : K_COL1_32];
  const size_t lds = sizeof(T) == 8 ? L.lds_col1_64 : L.lds_col1_32;
  cx<T>* sp = static_cast<cx<T>*>(spec);
  // the first engine variant launched carries the step-length work-groups
  CgState* a = alpha_cg;
  auto go = [&](auto kernel) {
    launch_tiles(kernel, ntiles + (a ? L.b.nrve : 0), lds, L.s, L.b, sp, cg, a);
    a = nullptr;
  };
  // cells with FP32 pencil pairs (bit 3) run on the 8-point kernel in FP64
  if (L.eng[1] & (sizeof(T) == 8 ? 10 : 2)) go(&k_col_a1<T, INV, 8>);
  if constexpr (sizeof(T) == 4)
    if (L.eng[1] & 8) go(&k_col_a1<T, INV, 16>);
  if (L.eng[1] & 4) go(&k_col_a1<T, INV, 12>);
  if (L.eng[1] & 1) go(&k_col_a1<T, INV, 0>);
}

void launch_col_a1(int prec, bool inverse, const Launch& L, void* spec, const CgState* cg, CgState* alpha_cg) {
  if (prec == PREC_F64) {
    if (inverse)
      col_a1_t<double, true>(L, spec, cg, alpha_cg);
    else
      col_a1_t<double, false>(L, spec, cg, alpha_cg);
  } else {
    if (inverse)
      col_a1_t<float, true>(L, spec, cg, alpha_cg);
    else
      col_a1_t<float, false>(L, spec, cg, alpha_cg);
  }
}

template <typename T>
static void col_a0_t(const Launch& L, void* spec, const CgState* cg) {
  const int ntiles = L.nblk[sizeof(T) == 8 ? K_COL0_64 : K_COL0_32];
  const size_t lds = sizeof(T) == 8 ? L.lds_col0_64 : L.lds_col0_32;
  cx<T>* sp = static_cast<cx<T>*>(spec);
  const int eng8 = sizeof(T) == 8 ? 10 : 2;  // cells with FP32 pencil pairs (bit 3) run on the 8-point kernel in FP64
  if (L.nyq) {
    if (L.eng[0] & eng8) launch_tiles(&k_col_a0_project<T, 8, true>, ntiles, lds, L.s, L.b, sp, cg);
    if constexpr (sizeof(T) == 4)
      if (L.eng[0] & 8) launch_tiles(&k_col_a0_project<T, 16, true>, ntiles, lds, L.s, L.b, sp, cg);
    if (L.eng[0] & 4) launch_tiles(&k_col_a0_project<T, 12, true>, ntiles, lds, L.s, L.b, sp, cg);
    if (L.eng[0] & 1) launch_tiles(&k_col_a0_project<T, 0, true>, ntiles, lds, L.s, L.b, sp, cg);
    return;
  }
  if (L.eng[0] & eng8) launch_tiles(&k_col_a0_project<T, 8, false>, ntiles, lds, L.s, L.b, sp, cg);
  if constexpr (sizeof(T) == 4)
    if (L.eng[0] & 8) launch_tiles(&k_col_a0_project<T, 16, false>, ntiles, lds, L.s, L.b, sp, cg);
  if (L.eng[0] & 4) launch_tiles(&k_col_a0_project<T, 12, false>, ntiles, lds, L.s, L.b, sp, cg);
  if (L.eng[0] & 1) launch_tiles(&k_col_a0_project<T, 0, false>, ntiles, lds, L.s, L.b, sp, cg);
}

void launch_col_a0_project(int prec, const Launch& L, void* spec, const CgState* cg) {
  if (prec == PREC_F64)
    col_a0_t<double>(L, spec, cg);
  else
    col_a0_t<float>(L, spec, cg);
}

template <typename T, int MODE, typename TO, bool NTOP = true>
static void inv_a2_mode(const Launch& L, const cx<T>* spec, TO* out, TO* x, double scale, const CgState* cg) {
  const int ntiles = L.nblk[K_ROW];
  const size_t lds = sizeof(T) == 8 ? L.lds_row64 : L.lds_row32;
  if (L.eng[2] & 2) launch_tiles(&k_inv_a2<T, MODE, TO, 8, NTOP>, ntiles, lds, L.s, L.b, spec, out, x, scale, cg);
  if (L.eng[2] & 4) launch_tiles(&k_inv_a2<T, MODE, TO, 12, NTOP>, ntiles, lds, L.s, L.b, spec, out, x, scale, cg);
  if (L.eng[2] & 1) launch_tiles(&k_inv_a2<T, MODE, TO, 0, NTOP>, ntiles, lds, L.s, L.b, spec, out, x, scale, cg);
}

template <typename T, typename TO>
static void inv_a2_t(int mode, const Launch& L, const void* spec, void* out, void* x, double scale,
                     const CgState* cg) {
  const cx<T>* sp = static_cast<const cx<T>*>(spec);
  TO* to = static_cast<TO*>(out);
  TO* tx = static_cast<TO*>(x);
  switch (mode) {
    case INV_OUT:
      if (L.ntop)
        inv_a2_mode<T, INV_OUT, TO, true>(L, sp, to, tx, scale, cg);
      else
        inv_a2_mode<T, INV_OUT, TO, false>(L, sp, to, tx, scale, cg);
      break;
    case INV_CGR: inv_a2_mode<T, INV_CGR, TO>(L, sp, to, tx, scale, cg); break;
    default: inv_a2_mode<T, INV_RHS, TO>(L, sp, to, tx, scale, cg); break;
  }
}

void launch_inv_a2(int prec, int mode, const Launch& L, const void* spec, void* out_T, int out_prec, void* x_T,
                   double scale, const CgState* cg) {
  if (prec == PREC_F64) {
    if (out_prec == PREC_F64)
      inv_a2_t<double, double>(mode, L, spec, out_T, x_T, scale, cg);
    else
      inv_a2_t<double, float>(mode, L, spec, out_T, x_T, scale, cg);
  } else {
    inv_a2_t<float, float>(mode, L, spec, out_T, x_T, scale, cg);
  }
}

}  // namespace fftnk
