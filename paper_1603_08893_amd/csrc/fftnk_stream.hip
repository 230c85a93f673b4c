// Streaming kernels that measure the achievable HBM rate of the device: the
// ceiling against which the operator's passes are judged (each pass moves
// every byte of its working set once, so its best possible time is its bytes
// over the best streaming rate, not over the nominal peak).
//
// Four access patterns over arrays of `bytes` bytes: read (a sum per
// work-group), write (a fill), copy, and triad a = b + s c; lanes of 8 or 16
// bytes; normal or non-temporal loads and stores.  Every work-group owns one
// contiguous chunk of 256 x 64 bytes per array, each thread issuing all four
// (16-byte lanes) or eight (8-byte lanes) loads of its chunk before using any.
#include "fftnk_internal.h"
#include "fftnk.h"

namespace fftnk {
namespace {

constexpr int kChunk = kThreads * 64;  // bytes of one array per work-group

// vector types the non-temporal builtins accept
typedef double dvec2 __attribute__((ext_vector_type(2)));
template <typename V>
struct lane_of {
  typedef V type;
};
template <>
struct lane_of<double2> {
  typedef dvec2 type;
};

template <bool NT, typename V>
__device__ __forceinline__ V ld(const V* p) {
  if constexpr (NT) {
    typedef typename lane_of<V>::type L;
    const L v = __builtin_nontemporal_load(reinterpret_cast<const L*>(p));
    return *reinterpret_cast<const V*>(&v);
  } else {
    return *p;
  }
}
template <bool NT, typename V>
__device__ __forceinline__ void st(V* p, const V& v) {
  if constexpr (NT) {
    typedef typename lane_of<V>::type L;
    __builtin_nontemporal_store(*reinterpret_cast<const L*>(&v), reinterpret_cast<L*>(p));
  } else {
    *p = v;
  }
}

template <typename V>
__device__ __forceinline__ double lane_sum(const V& v);
template <>
__device__ __forceinline__ double lane_sum<double>(const double& v) { return v; }
template <>
__device__ __forceinline__ double lane_sum<double2>(const double2& v) { return v.x + v.y; }

template <typename V>
__device__ __forceinline__ V splat(double s);
template <>
__device__ __forceinline__ double splat<double>(double s) { return s; }
template <>
__device__ __forceinline__ double2 splat<double2>(double s) { return double2{s, s}; }

template <typename V, bool NT>
__global__ __launch_bounds__(kThreads) void k_stream_read(const V* __restrict__ a, long long nv,
                                                          double* __restrict__ out) {
  constexpr int U = 64 / sizeof(V);
  const long long base = (long long)blockIdx.x * (kThreads * U) + threadIdx.x;
  V v[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const long long i = base + (long long)u * kThreads;
    v[u] = i < nv ? ld<NT>(a + i) : splat<V>(0.0);
  }
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < U; ++u) s += lane_sum<V>(v[u]);
  // a partial per work-group (fixed order: lanes, then waves through LDS)
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  __shared__ double w[kThreads / 64];
  if ((threadIdx.x & 63) == 0) w[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < kThreads / 64; ++k) t += w[k];
    out[blockIdx.x] = t;
  }
}

template <typename V, bool NT>
__global__ __launch_bounds__(kThreads) void k_stream_write(V* __restrict__ a, long long nv, double val) {
  constexpr int U = 64 / sizeof(V);
  const long long base = (long long)blockIdx.x * (kThreads * U) + threadIdx.x;
  const V x = splat<V>(val);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const long long i = base + (long long)u * kThreads;
    if (i < nv) st<NT>(a + i, x);
  }
}

template <typename V, bool NT>
__global__ __launch_bounds__(kThreads) void k_stream_copy(V* __restrict__ a, const V* __restrict__ b, long long nv) {
  constexpr int U = 64 / sizeof(V);
  const long long base = (long long)blockIdx.x * (kThreads * U) + threadIdx.x;
  V v[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const long long i = base + (long long)u * kThreads;
    if (i < nv) v[u] = ld<NT>(b + i);
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const long long i = base + (long long)u * kThreads;
    if (i < nv) st<NT>(a + i, v[u]);
  }
}

template <typename V, bool NT>
__global__ __launch_bounds__(kThreads) void k_stream_triad(V* __restrict__ a, const V* __restrict__ b,
                                                           const V* __restrict__ c, double s, long long nv) {
  constexpr int U = 64 / sizeof(V);
  const long long base = (long long)blockIdx.x * (kThreads * U) + threadIdx.x;
  V x[U], y[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const long long i = base + (long long)u * kThreads;
    if (i < nv) {
      x[u] = ld<NT>(b + i);
      y[u] = ld<NT>(c + i);
    }
  }
  const V sv = splat<V>(s);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const long long i = base + (long long)u * kThreads;
    if (i < nv) st<NT>(a + i, V(x[u] + sv * y[u]));
  }
}

template <typename V, bool NT>
void launch_stream(int kind, void* dst, const void* s1, const void* s2, long long nv, int blocks, hipStream_t st) {
  const dim3 grid(blocks), block(kThreads);
  switch (kind) {
    case FFTNK_STREAM_READ:
      k_stream_read<V, NT><<<grid, block, 0, st>>>(static_cast<const V*>(s1), nv, static_cast<double*>(dst));
      break;
    case FFTNK_STREAM_WRITE:
      k_stream_write<V, NT><<<grid, block, 0, st>>>(static_cast<V*>(dst), nv, 1.0);
      break;
    case FFTNK_STREAM_COPY:
      k_stream_copy<V, NT><<<grid, block, 0, st>>>(static_cast<V*>(dst), static_cast<const V*>(s1), nv);
      break;
    default:
      k_stream_triad<V, NT><<<grid, block, 0, st>>>(static_cast<V*>(dst), static_cast<const V*>(s1),
                                                   static_cast<const V*>(s2), 0.5, nv);
      break;
  }
}

}  // namespace
}  // namespace fftnk

extern "C" int fftnk_stream(int kind, int lane_bytes, void* dst, const void* src1, const void* src2, size_t bytes,
                            int reps, void* hip_stream, double* ms_host) {
  using namespace fftnk;
  const bool nt = (kind & FFTNK_STREAM_NONTEMPORAL) != 0;
  kind &= ~FFTNK_STREAM_NONTEMPORAL;
  if (kind < FFTNK_STREAM_READ || kind > FFTNK_STREAM_TRIAD) return FFTNK_EINVAL;
  if (lane_bytes != 8 && lane_bytes != 16) return FFTNK_EINVAL;
  if (bytes == 0 || bytes % (size_t)lane_bytes || reps < 1 || reps > 10000 || !ms_host) return FFTNK_EINVAL;
  const bool need1 = kind != FFTNK_STREAM_WRITE, need2 = kind == FFTNK_STREAM_TRIAD;
  if (!dst || (need1 && !src1) || (need2 && !src2)) return FFTNK_EINVAL;
  const long long blocks = (long long)((bytes + kChunk - 1) / kChunk);
  if (blocks > 0x7fffffffLL) return FFTNK_EINVAL;
  const long long nv = (long long)(bytes / (size_t)lane_bytes);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  auto go = [&]() {
    if (lane_bytes == 8)
      nt ? launch_stream<double, true>(kind, dst, src1, src2, nv, (int)blocks, st)
         : launch_stream<double, false>(kind, dst, src1, src2, nv, (int)blocks, st);
    else
      nt ? launch_stream<double2, true>(kind, dst, src1, src2, nv, (int)blocks, st)
         : launch_stream<double2, false>(kind, dst, src1, src2, nv, (int)blocks, st);
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess) return FFTNK_EHIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return FFTNK_EHIP;
  }
  int status = FFTNK_OK;
  go();  // warm-up (first-touch, code load)
  if (hipGetLastError() != hipSuccess || hipEventRecord(e0, st) != hipSuccess) status = FFTNK_EHIP;
  if (status == FFTNK_OK) {
    for (int k = 0; k < reps; ++k) go();
    if (hipGetLastError() != hipSuccess || hipEventRecord(e1, st) != hipSuccess ||
        hipEventSynchronize(e1) != hipSuccess)
      status = FFTNK_EHIP;
  }
  float ms = 0.0f;
  if (status == FFTNK_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) status = FFTNK_EHIP;
  if (status == FFTNK_OK) *ms_host = (double)ms / reps;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return status;
}
