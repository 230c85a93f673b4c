// Device helpers of libfftnk (gfx950): complex arithmetic, the two FFT engines,
// deterministic block reductions, the work-group -> RVE map and the
// St. Venant-Kirchhoff constitutive law.  Included by the kernel sources only.
#pragma once

#include "fftnk_internal.h"

namespace fftnk {

// Launch metadata that a kernel only reads (grids, start tables, masks, uniform
// tensors, and the CG scalars, which only other launches write) is read through
// the constant address space: uniform reads of it become scalar loads, also in
// the tile loops of kernels that store to global memory (where the compiler
// could not otherwise rule out aliasing and would use vector loads).
template <typename T>
using cptr_t = const __attribute__((address_space(4))) T*;
template <typename T>
__device__ __forceinline__ cptr_t<T> cptr(const T* p) {
  return (cptr_t<T>)p;
}
__device__ __forceinline__ const __attribute__((address_space(4))) Grid& grid_of(const Batch& B, int rv) {
  return *cptr(B.grids + rv);
}

// p advanced by b bytes.  With p uniform and b a 32-bit lane offset the access
// compiles to a scalar base plus one offset register (no 64-bit lane address).
template <typename T>
__device__ __forceinline__ T* byte_off(T* p, unsigned b) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(p) + b);
}
template <typename T>
__device__ __forceinline__ const T* byte_off(const T* p, unsigned b) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + b);
}

// Streaming accesses of the operator passes.  Fields that one pass reads or
// writes once and that are not touched again before the data would be evicted
// anyway (the Krylov vectors r, p, x in pass 1, the residual in pass 5, the
// direction and the result of a single operator application) use
// non-temporal loads and stores.  With the 36 read and 27 write streams of
// pass 1 in flight per voxel, the normal replacement policy held the HBM rate
// about 10 % below the non-temporal one (128^3 FP64 and FP32, 192^3, 256^3).
// The linearisation point F and the spectrum stay normal (both measured slower
// non-temporally), and so does the FP32 residual of pass 5: at 128^3 the FP32
// fields fit the last-level cache, where pass 1 of the next iteration finds r.
// Bit k of the policy switches the accesses of class k (per element size).
#ifndef FFTNK_NT_POLICY64
#define FFTNK_NT_POLICY64 (1 | 4 | 16 | 32 | 64 | 128)
#endif
#ifndef FFTNK_NT_POLICY32
#define FFTNK_NT_POLICY32 (1 | 4 | 64 | 128)
#endif
enum {
  NT_P1_LOAD_VEC = 1,   // pass 1: loads of r, the previous p, x
  NT_P1_LOAD_F = 2,     // pass 1: loads of the linearisation point F
  NT_P1_STORE_VEC = 4,  // pass 1: stores of x and p
  NT_P1_STORE_SPEC = 8, // pass 1: stores of the half spectrum
  NT_P5_LOAD_R = 16,    // pass 5 (CG): loads of r
  NT_P5_STORE_R = 32,   // pass 5 (CG): stores of r
  NT_OP_LOAD_P = 64,    // pass 1 (operator): loads of the direction
  NT_OP_STORE_OUT = 128 // pass 5 (operator, projection): stores of the result
};
template <typename T>
__host__ __device__ constexpr int nt_policy() {
  return sizeof(T) == 8 ? FFTNK_NT_POLICY64 : FFTNK_NT_POLICY32;
}

template <int CLASS, typename T>
__device__ __forceinline__ T ld_stream(const T* p) {
  if constexpr ((nt_policy<T>() & CLASS) != 0) {
    return __builtin_nontemporal_load(p);
  } else {
    return *p;
  }
}
template <int CLASS, typename T>
__device__ __forceinline__ void st_stream(T* p, T v) {
  if constexpr ((nt_policy<T>() & CLASS) != 0) {
    __builtin_nontemporal_store(v, p);
  } else {
    *p = v;
  }
}
// the same where a launch decides: NT false keeps ordinary accesses (operator
// applications on cells whose fields fit the last-level cache, Launch::ntop)
template <bool NT, int CLASS, typename T>
__device__ __forceinline__ T ld_stream_if(const T* p) {
  if constexpr (NT) return ld_stream<CLASS>(p);
  else return *p;
}
template <bool NT, int CLASS, typename T>
__device__ __forceinline__ void st_stream_if(T* p, T v) {
  if constexpr (NT) st_stream<CLASS>(p, v);
  else *p = v;
}

// ---------------------------------------------------------------------------
// complex arithmetic
// ---------------------------------------------------------------------------
template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T x, y;
};

// two complex values adjacent in memory (one 4 sizeof(T)-byte access)
template <typename T>
struct alignas(4 * sizeof(T)) cx2 {
  cx<T> a, b;
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
// W_n^e from the forward table (exp(-2 pi i e / n)); conjugated for the inverse
template <typename T>
__device__ __forceinline__ cx<T> twid(const cx<T>* tw, int e, bool inv) {
  cx<T> w = tw[lpad(e)];
  if (inv) w.y = -w.y;
  return w;
}

// ---------------------------------------------------------------------------
// small DFTs in registers: v[q] <- sum_r v[r] W_R^{rq}, W_R = exp(-+2 pi i / R)
// ---------------------------------------------------------------------------
template <typename T, int R>
struct SmallDft {
  // any radix through the length-n twiddle table (W_R^e = W_n^{e n/R})
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

// 3-point DFT in place: X1,2 = a0 - (a1 + a2)/2 -+ (sqrt(3)/2) i (a1 - a2)
// (signs for the forward transform; the inverse conjugates W_3).
template <typename T>
__device__ __forceinline__ void dft3(cx<T>& a0, cx<T>& a1, cx<T>& a2, bool inv) {
  const T s = (T)0.86602540378443864676;  // sqrt(3) / 2
  const cx<T> t1 = a1 + a2;
  const cx<T> t2 = a0 - cscale(t1, (T)0.5);
  const cx<T> t3 = cscale(rot(a1 - a2, inv), s);
  a0 = a0 + t1;
  a1 = t2 + t3;
  a2 = t2 - t3;
}

// 12-point DFT as 3 x 4: with r = r1 + 3 r2 and q = 4 q1 + q2,
// X[q] = sum_r1 W_3^{r1 q1} (W_12^{r1 q2} B_r1[q2]), B_r1 the 4-point DFT of
// a[r1 + 3 r2] over r2; outputs in natural order.
template <typename T>
struct SmallDft<T, 12> {
  __device__ __forceinline__ static void run(cx<T>* v, const cx<T>*, int, bool inv) {
    const T c = (T)0.86602540378443864676, h = (T)0.5;  // cos 30 deg, sin 30 deg
    const T sg = inv ? (T)1 : (T)-1;                    // sign of the imaginary parts of W_12^k
    cx<T> b[3][4];
#pragma unroll
    for (int r1 = 0; r1 < 3; ++r1) {
      b[r1][0] = v[r1];
      b[r1][1] = v[r1 + 3];
      b[r1][2] = v[r1 + 6];
      b[r1][3] = v[r1 + 9];
      dft4(b[r1][0], b[r1][1], b[r1][2], b[r1][3], inv);
    }
    // W_12^1, W_12^2, W_12^3 on r1 = 1; W_12^2, W_12^4, W_12^6 on r1 = 2
    b[1][1] = cmul(b[1][1], cx<T>{c, sg * h});
    b[1][2] = cmul(b[1][2], cx<T>{h, sg * c});
    b[1][3] = rot(b[1][3], inv);
    b[2][1] = cmul(b[2][1], cx<T>{h, sg * c});
    b[2][2] = cmul(b[2][2], cx<T>{-h, sg * c});
    b[2][3] = cx<T>{-b[2][3].x, -b[2][3].y};
#pragma unroll
    for (int q2 = 0; q2 < 4; ++q2) {
      dft3(b[0][q2], b[1][q2], b[2][q2], inv);
      v[q2] = b[0][q2];
      v[4 + q2] = b[1][q2];
      v[8 + q2] = b[2][q2];
    }
  }
};

// ---------------------------------------------------------------------------
// LDS engine (any length): Stockham autosort stages on `npen` pencils of
// length n held in LDS, element e of pencil m at m*sp + e*se.  Ns is the
// product of the previous radices.  Butterfly j (0 <= j < n/R) reads
// e = j + r n/R, applies W_{Ns R}^{k r} (k = j mod Ns), does an R-point DFT and
// writes e = (j - k) R + k + r Ns.  pen_fast selects which index consecutive
// threads walk (pencils for column tiles, butterflies for row tiles).
// ---------------------------------------------------------------------------
template <typename T, int R>
__device__ __forceinline__ void stage_lds(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst, int n, int Ns, int npen, int sp,
                          int se, const cx<T>* tw, bool inv, bool pen_fast) {
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

// Stage for a prime radix R >= 11.  The outputs of a butterfly come in pairs
// (q, R - q) that share their terms: with the stage-twiddled inputs
// y_r = x[j + r n/R] W_n^{k r n/(Ns R)} and, for r = 1 .. (R-1)/2,
// a_r = y_r + y_{R-r}, b_r = y_r - y_{R-r} and theta = 2 pi r q / R,
//   X_0     = y_0 + sum_r a_r
//   X_q     = y_0 + sum_r a_r cos(theta) -/+ i sum_r b_r sin(theta)
//   X_{R-q} = y_0 + sum_r a_r cos(theta) +/- i sum_r b_r sin(theta)
// (upper signs forward, W = exp(-2 pi i / R)): half the multiply-adds of the
// direct sum, and each input is read once per group of kPrimePairs output
// pairs instead of once per output.  A work item is (butterfly, group of
// pairs); consecutive items walk the butterflies, so the lanes of a wave read
// the same cos / sin entries (LDS broadcasts).  The cos / sin of theta are
// W_R^m = W_n^{m n/R} from the stage's twiddle table.
constexpr int kPrimePairs = 5;
template <typename T>
__device__ __forceinline__ void stage_lds_prime(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst, int n, int Ns,
                                                int R, int npen, int sp, int se, const cx<T>* tw, bool inv,
                                                bool pen_fast) {
  constexpr int C = kPrimePairs;
  const int nbf = n / R, half = (R - 1) / 2;
  const int ngrp = (half + C - 1) / C;
  const int nb = nbf * npen;
  const int total = nb * ngrp;
  const int tws = n / (Ns * R);
  const T sg = inv ? (T)1 : (T)-1;  // X_q = U + sg i V
  for (int it = threadIdx.x; it < total; it += kThreads) {
    const int grp = it / nb, bb = it - grp * nb;
    int m, j;
    if (pen_fast) {
      j = bb / npen;
      m = bb - j * npen;
    } else {
      m = bb / nbf;
      j = bb - m * nbf;
    }
    const int k = j % Ns;
    const int ek = k * tws;  // stage twiddle of input r: W_n^{ek r}
    const cx<T>* s = src + m * sp;
    const cx<T> y0 = s[j * se];
    const int q0 = 1 + grp * C;
    cx<T> U[C], V[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      U[c] = y0;
      V[c] = cx<T>{(T)0, (T)0};
    }
    cx<T> sum_a = y0;
    int ep = ek;                                      // (ek r) mod n
    int em = (int)(((long long)ek * (R - 1)) % n);  // (ek (R - r)) mod n
    for (int r = 1; r <= half; ++r) {
      cx<T> yp = s[(j + r * nbf) * se], ym = s[(j + (R - r) * nbf) * se];
      if (k != 0) {
        yp = cmul(yp, twid(tw, ep, inv));
        ym = cmul(ym, twid(tw, em, inv));
      }
      ep += ek;
      if (ep >= n) ep -= n;
      em -= ek;
      if (em < 0) em += n;
      const cx<T> a = yp + ym, d = yp - ym;
      sum_a = sum_a + a;
      int e = (r * q0) % R;  // r q mod R for q = q0 + c
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const cx<T> w = tw[lpad(e * nbf)];  // (cos theta, -sin theta)
        U[c] = U[c] + cscale(a, w.x);
        V[c] = V[c] - cscale(d, w.y);
        e += r;
        if (e >= R) e -= R;
      }
    }
    cx<T>* dd = dst + m * sp;
    const int base = (j - k) * R + k;
    if (grp == 0) dd[base * se] = sum_a;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int q = q0 + c;
      if (q > half) break;
      const cx<T> iv{-sg * V[c].y, sg * V[c].x};  // sg i V
      dd[(base + q * Ns) * se] = U[c] + iv;
      dd[(base + (R - q) * Ns) * se] = U[c] - iv;
    }
  }
}

// Full 1-D transform of npen pencils; buffers a (input) and b (scratch)
// ping-pong.  Returns the buffer holding the result.  The caller synchronises
// before (input written); the routine synchronises after every stage.
template <typename T, typename PL>
__device__ __forceinline__ cx<T>* fft_lds(cx<T>* a, cx<T>* b, const PL& pl, int npen, int sp, int se, const cx<T>* tw,
                          bool inv, bool pen_fast) {
  int Ns = 1;
  for (int s = 0; s < pl.nstages; ++s) {
    const int R = pl.radix[s];
    switch (R) {
      case 2: stage_lds<T, 2>(a, b, pl.n, Ns, npen, sp, se, tw, inv, pen_fast); break;
      case 3: stage_lds<T, 3>(a, b, pl.n, Ns, npen, sp, se, tw, inv, pen_fast); break;
      case 4: stage_lds<T, 4>(a, b, pl.n, Ns, npen, sp, se, tw, inv, pen_fast); break;
      case 5: stage_lds<T, 5>(a, b, pl.n, Ns, npen, sp, se, tw, inv, pen_fast); break;
      case 7: stage_lds<T, 7>(a, b, pl.n, Ns, npen, sp, se, tw, inv, pen_fast); break;
      case 8: stage_lds<T, 8>(a, b, pl.n, Ns, npen, sp, se, tw, inv, pen_fast); break;
      default: stage_lds_prime<T>(a, b, pl.n, Ns, R, npen, sp, se, tw, inv, pen_fast); break;
    }
    __syncthreads();
    cx<T>* t = a;
    a = b;
    b = t;
    Ns *= R;
  }
  return a;
}

// ---------------------------------------------------------------------------
// Register-resident engine, specialised at compile time for every length so
// that all index arithmetic is shifts and constants: P = 8 points per thread
// for powers of two 8 <= n <= kMaxLen (radices 8 / 4 / 2), P = 12 for
// n = 3 2^k, 12 <= n <= 192 (a radix-12 stage, then radices 4 / 2).
// A pencil is split over Tp = n / P threads; thread t holds
// v[q] = x[t + Tp q], q < P, for the whole transform.  In every Stockham
// stage the butterflies of thread t are j = t + k Tp (k < P / R) and their
// inputs are exactly its own registers v[k + r P/R]; only the outputs move,
// through one LDS exchange per stage, and the outputs of the last stage land in
// natural order on the same register slots, so loads from and stores to global
// memory need no LDS.  Exchange layouts: ROW == false, pencils interleaved
// (element e of the thread's pencil at xl[e * ES], ES = kThreads / Tp pencils,
// consecutive lanes own consecutive pencils); ROW == true, one unit-stride line
// per pencil (element e at xl[lpad(e)], the slot spans padded_len(n) entries).
// The radix sequence splits log2 n into ceil(log2 n / 3) near-equal stages,
// larger radices first.  All threads of the work-group must call it (it
// contains barriers).
// ---------------------------------------------------------------------------
constexpr int ct_log2(int n) { return n <= 1 ? 0 : 1 + ct_log2(n >> 1); }
// Radix plan of the register engine.  P = 8 (n = 2^k, 8 <= n <= 256): log2 n
// split into ceil(log2 n / 3) near-equal power-of-two stages, larger first.
// P = 12 (n = 3 2^k, 12 <= n <= 192): one radix-12 stage, then radix 4 stages
// (and one radix 2 for an odd power).  Every radix divides P.
template <int P>
constexpr int ct_nstages(int n) {
  if constexpr (P == 8)
    return (ct_log2(n) + 2) / 3;
  else
    return 1 + (ct_log2(n / 12) + 1) / 2;
}
template <int P>
constexpr int ct_radix(int n, int s) {
  if constexpr (P == 8) {
    return 1 << (ct_log2(n) / ct_nstages<8>(n) + (s < ct_log2(n) % ct_nstages<8>(n) ? 1 : 0));
  } else {
    return s == 0 ? 12 : ((s < 1 + ct_log2(n / 12) / 2) ? 4 : 2);
  }
}
template <int P>
constexpr int ct_span(int n, int s) { return s == 0 ? 1 : ct_span<P>(n, s - 1) * ct_radix<P>(n, s - 1); }

template <int N, int P, bool ROW>
__device__ __forceinline__ int xslot(int e) {
  if constexpr (ROW)
    return lpad(e);
  else
    return e * (kThreads * P / N);
}

template <typename T, int N, int P, bool ROW, int S>
__device__ __forceinline__ void reg_stages(cx<T> (&v)[P], int t, const cx<T>* tw, bool inv, cx<T>* xl) {
  if constexpr (S < ct_nstages<P>(N)) {
    constexpr int R = ct_radix<P>(N, S), NS = ct_span<P>(N, S), Tp = N / P, B = P / R, TWS = N / (NS * R);
    static_assert(P % R == 0, "every radix divides the points per thread");
    constexpr bool LAST = S + 1 == ct_nstages<P>(N);
#pragma unroll
    for (int k = 0; k < B; ++k) {
      cx<T> a[R];
#pragma unroll
      for (int r = 0; r < R; ++r) a[r] = v[k + r * B];
      const int j = t + k * Tp;
      const int kk = (NS & (NS - 1)) == 0 ? (j & (NS - 1)) : (j % NS);
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) a[r] = cmul(a[r], twid(tw, kk * (r * TWS), inv));
      }
      SmallDft<T, R>::run(a, tw, N, inv);
      if constexpr (LAST) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[k + r * B] = a[r];
      } else {
        const int base = (j - kk) * R + kk;
#pragma unroll
        for (int r = 0; r < R; ++r) xl[xslot<N, P, ROW>(base + r * NS)] = a[r];
      }
    }
    if constexpr (!LAST) {
      __syncthreads();
#pragma unroll
      for (int q = 0; q < P; ++q) v[q] = xl[xslot<N, P, ROW>(t + Tp * q)];
      __syncthreads();
      reg_stages<T, N, P, ROW, S + 1>(v, t, tw, inv, xl);
    }
  }
}

// Transform of length n with P points per thread: P = 8 for n a power of two in
// [8, kMaxRegLen], P = 12 for n = 3 2^k in [12, 192]; t in [0, n / P).
template <typename T, bool ROW, int P>
__device__ __forceinline__ void reg_fft(cx<T> (&v)[P], int n, int t, const cx<T>* tw, bool inv, cx<T>* xl) {
  static_assert(kMaxRegLen == 256, "length dispatch covers 8..256");
  if constexpr (P == 8) {
    switch (n) {
      case 8: reg_stages<T, 8, 8, ROW, 0>(v, t, tw, inv, xl); break;
      case 16: reg_stages<T, 16, 8, ROW, 0>(v, t, tw, inv, xl); break;
      case 32: reg_stages<T, 32, 8, ROW, 0>(v, t, tw, inv, xl); break;
      case 64: reg_stages<T, 64, 8, ROW, 0>(v, t, tw, inv, xl); break;
      case 128: reg_stages<T, 128, 8, ROW, 0>(v, t, tw, inv, xl); break;
      default: reg_stages<T, 256, 8, ROW, 0>(v, t, tw, inv, xl); break;
    }
  } else {
    static_assert(P == 12, "register engine: 8 or 12 points per thread");
    switch (n) {
      case 12: reg_stages<T, 12, 12, ROW, 0>(v, t, tw, inv, xl); break;
      case 24: reg_stages<T, 24, 12, ROW, 0>(v, t, tw, inv, xl); break;
      case 48: reg_stages<T, 48, 12, ROW, 0>(v, t, tw, inv, xl); break;
      case 96: reg_stages<T, 96, 12, ROW, 0>(v, t, tw, inv, xl); break;
      default: reg_stages<T, 192, 12, ROW, 0>(v, t, tw, inv, xl); break;
    }
  }
}

template <typename T>
__device__ __forceinline__ const cx<T>* table_of(const Batch& B) {
  return reinterpret_cast<const cx<T>*>(sizeof(T) == 8 ? B.tw64 : B.tw32);
}

template <typename T>
__device__ __forceinline__ void load_twiddles(cx<T>* dst, const Batch& B, int off, int n) {
  const cx<T>* src = table_of<T>(B) + off;
  for (int i = threadIdx.x; i < n; i += kThreads) dst[lpad(i)] = src[i];
}


// ---------------------------------------------------------------------------
// work-group -> RVE (binary search in the launch kind's start table)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int find_rve(const Batch& B, int kind, int b, int& local) {
  const auto s = cptr(B.starts + kind * (B.nrve + 1));
  int lo = 0, hi = B.nrve;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (s[mid] <= b)
      lo = mid;
    else
      hi = mid;
  }
  local = b - s[lo];
  return lo;
}

__device__ __forceinline__ int rve_blocks(const Batch& B, int kind, int r) {
  const auto s = cptr(B.starts + kind * (B.nrve + 1));
  return s[r + 1] - s[r];
}

// skip rule of a launch: CG launches skip RVEs whose CG is done, Newton-level
// launches skip RVEs that have finished the increment
__device__ __forceinline__ bool skip_rve(const Batch& B, const CgState* cg, int r) {
  if (cg) return cptr(cg)[r].done != 0;
  return B.active && cptr(B.active)[r] == 0;
}

// ---------------------------------------------------------------------------
// deterministic block reduction (wave shuffles, then the waves in order)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

template <int K>
__device__ __forceinline__ void block_sums(double (&v)[K], double* out /* K results, thread 0 */) {
  __shared__ double red[kThreads / 64][K];
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

__device__ __forceinline__ double* pslot(const Batch& B, int slot) { return B.partials + (long long)slot * B.pstride; }

// Fixed-order sum of partials[lo, hi) by one work-group; result in every thread.
// Eight independent accumulators per thread keep eight loads in flight.
__device__ __forceinline__ double reduce_range(const double* part, int lo, int hi) {
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int i = lo + threadIdx.x;
  for (; i + 7 * kThreads < hi; i += 8 * kThreads) {
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += part[i + u * kThreads];
  }
  for (; i < hi; i += kThreads) a[0] += part[i];
  double s[1] = {((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]))};
  double res[1];
  block_sums<1>(s, res);
  __shared__ double bc;
  if (threadIdx.x == 0) bc = res[0];
  __syncthreads();
  return bc;
}

// The CG step length of RVE rv by one work-group (its whole block), right
// after the first pass: alpha = <r, r> / <p, A p>.  It runs as extra work-
// groups of the second pass's launch (the middle passes do not use alpha;
// the last pass does).  With A = G K and
// G the orthogonal projection (symmetric, p in its range as every Krylov
// direction is), <p, A p> = <G p, K p> = <p, K p>: the first pass sums it from
// p and K p in registers, so the last pass never reads p again.
//
// Bookkeeping of the deferred x updates: iteration k's first pass applied
// the window of directions before k when k mod W = 0 (x_lo = k); alpha_k goes
// to its slot of the history and term k becomes due (x_hi = k + 1) unless the
// iteration breaks down.
__device__ __forceinline__ int kstart(const Batch& B, int kind, int r) { return B.starts[kind * (B.nrve + 1) + r]; }

__device__ __forceinline__ void cg_alpha_group(const Batch& B, CgState* cg, int rv) {
  CgState& s = cg[rv];
  if (s.done) return;
  if (threadIdx.x == 0 && s.iter > 0 && s.iter % B.xwin == 0) s.x_lo = s.iter;
  if (s.method != KRYLOV_CG) {  // fixed coefficients: the step of the recurrence
    if (threadIdx.x == 0) {
      s.alpha = s.method == KRYLOV_CHEBYSHEV ? s.gam : 2.0 / (s.lo + s.hi);
      s.ahist[s.iter % B.xwin] = s.alpha;
      s.x_hi = s.iter + 1;
    }
    return;
  }
  const double pw = reduce_range(pslot(B, SLOT_PW), kstart(B, K_ROW1, rv), kstart(B, K_ROW1, rv + 1));
  if (threadIdx.x == 0) {
    s.pw = pw;
    if (!(pw > 0.0) || !isfinite(pw)) {
      // With the stagnation guard on (FP32 Krylov vectors), a non-positive
      // curvature once the residual is near the FP32 rounding floor (relative
      // residual <= 1e-5, after the first iteration) means the direction is
      // round-off noise: stop and keep the last iterate, as for stagnation; the
      // FP64 Newton residual corrects the inexact update.  Otherwise it is a
      // breakdown (indefinite tangent), as in FP64.
      s.status = (s.stall_limit > 0 && s.iter > 0 && isfinite(pw) && s.rr <= 1e-10 * s.bb) ? ST_OK
                                                                                         : ST_CG_BREAKDOWN;
      s.done = 1;
      s.alpha = 0.0;
      s.x_hi = s.iter;  // this iteration's direction is not applied
    } else {
      s.alpha = s.rr / pw;
      s.ahist[s.iter % B.xwin] = s.alpha;
      s.x_hi = s.iter + 1;
    }
  }
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

// v: global voxel index (over all RVEs)
__device__ __forceinline__ void material_at(const Material& mat, long long v, double& lam, double& mu) {
  const int ph = mat.phase[v];
  const double* row = mat.table + 4 * ph;
  mu = mat.mu_field ? mat.mu_field[v] : row[1];
  lam = row[0] - 2.0 * mu / 3.0;
}

__device__ __forceinline__ int signed_freq(int k, int n) { return 2 * k > n ? k - n : k; }

}  // namespace fftnk
