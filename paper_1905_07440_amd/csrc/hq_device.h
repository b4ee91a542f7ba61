// Device-side helpers of libhq: the counter-based generator, MFMA fragment
// types and small wave/block reductions.  gfx950 (CDNA4), wave64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hq {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11): 10 rounds, multipliers M0/M1, Weyl
// key increments W0/W1.  Counter (chain, sweep, slot, kind), key (seed, 0).
// ---------------------------------------------------------------------------
struct Philox4 { uint64_t w[4]; };

__host__ __device__ inline void mulhilo64(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
#if defined(__HIP_DEVICE_COMPILE__)
  lo = a * b;
  hi = __umul64hi(a, b);
#else
  unsigned __int128 p = (unsigned __int128)a * b;
  lo = (uint64_t)p;
  hi = (uint64_t)(p >> 64);
#endif
}

__host__ __device__ inline Philox4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                                  uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t hi0, lo0, hi1, lo1;
    mulhilo64(M0, c0, hi0, lo0);
    mulhilo64(M1, c2, hi1, lo1);
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += W0; k1 += W1;
  }
  Philox4 out;
  out.w[0] = c0; out.w[1] = c1; out.w[2] = c2; out.w[3] = c3;
  return out;
}

// top 53 bits as a double in [0, 1)
__host__ __device__ inline double u53(uint64_t w) {
  return (double)(w >> 11) * (1.0 / 9007199254740992.0);
}

enum { KIND_LOCAL = 0, KIND_GLOBAL = 1, KIND_INIT = 2, KIND_NN = 3, KIND_CUMULATIVE = 4,
       KIND_COUPLING = 5, KIND_NN_GLOBAL = 6, KIND_SCAN = 7 };

// ---------------------------------------------------------------------------
// MFMA 16x16x4 wrappers.  Operand layout (measured on gfx950):
//   A (16x4):  lane l holds A[l % 16][l / 16]
//   B (4x16):  lane l holds B[l / 16][l % 16]
//   D (16x16): lane l, element v holds D[frag_row(l, v)][l % 16] with
//              frag_row = 4*v + l/16 for f64 and 4*(l/16) + v for f32.
// ---------------------------------------------------------------------------
template <typename T> __device__ inline int frag_row(int lane, int v);
template <> __device__ inline int frag_row<double>(int lane, int v) { return 4 * v + (lane >> 4); }
template <> __device__ inline int frag_row<float>(int lane, int v) { return 4 * (lane >> 4) + v; }
template <typename T> struct Frag;
template <> struct Frag<double> { typedef d4 type; };
template <> struct Frag<float> { typedef f4 type; };

__device__ inline d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4 mfma16(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
template <typename T>
__device__ inline T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
// sum over groups of W consecutive lanes (W a power of two <= 64)
template <int W, typename T>
__device__ inline T group_sum(T v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// block-wide sum of one double per thread, deterministic order; all threads
// get the result.  scratch: >= NT/64 doubles of LDS.
template <int NT>
__device__ inline double block_sum(double v, double* scratch) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) scratch[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < NT / 64; ++k) s += scratch[k];
  return s;
}
template <int NT>
__device__ inline double block_max(double v, double* scratch) {
  v = wave_max(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) scratch[w] = v;
  __syncthreads();
  double s = scratch[0];
#pragma unroll
  for (int k = 1; k < NT / 64; ++k) s = fmax(s, scratch[k]);
  return s;
}

// dst(e, src(e)) for e in [0, count) over NT threads, with UNR loads of each
// thread in flight before the first store (a copy loop that waited for every
// load on its own would be bound by memory latency, not bandwidth)
template <int NT, int UNR, typename T, typename Src, typename Dst>
__device__ inline void batched_copy(int count, Src src, Dst dst) {
  for (int base = 0; base < count; base += NT * UNR) {
    T v[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int e = base + u * NT + (int)threadIdx.x;
      v[u] = (e < count) ? src(e) : T(0);
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int e = base + u * NT + (int)threadIdx.x;
      if (e < count) dst(e, v[u]);
    }
  }
}

// Raw buffer loads and stores: an element's address is a 32-bit byte offset
// into a resource (base, size); an offset at or past the size reads 0 and
// drops the store, so a masked offset replaces a bounds branch.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr unsigned BUF_WORD3 = 0x00020000u;   // raw buffer, 32-bit data format (gfx9)
constexpr unsigned BUF_OUTSIDE = 0x80000000u;  // an offset no resource here reaches
// a double through the 64-bit buffer operations, word by word (a bit cast of an
// accumulator element straight to the two-word type stored wrong values for
// every element but the first)
__device__ inline double buf_load_f64(__amdgpu_buffer_rsrc_t r, unsigned off) {
  const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
  return __builtin_bit_cast(double, ((unsigned long long)w.y << 32) | w.x);
}
__device__ inline void buf_store_f64(double v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  u32x2 w;
  w.x = (unsigned)u;
  w.y = (unsigned)(u >> 32);
  __builtin_amdgcn_raw_buffer_store_b64(w, r, off, 0, 0);
}
__device__ inline float buf_load_f32(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ inline void buf_store_f32(float v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}
__device__ inline double buf_load(__amdgpu_buffer_rsrc_t r, unsigned off, double*) { return buf_load_f64(r, off); }
__device__ inline float buf_load(__amdgpu_buffer_rsrc_t r, unsigned off, float*) { return buf_load_f32(r, off); }
__device__ inline void buf_store(double v, __amdgpu_buffer_rsrc_t r, unsigned off) { buf_store_f64(v, r, off); }
__device__ inline void buf_store(float v, __amdgpu_buffer_rsrc_t r, unsigned off) { buf_store_f32(v, r, off); }

// a buffer resource over bytes from p, with p made wave-uniform first: a
// resource that the compiler keeps in vector registers (a select between two
// of them, say) puts every load through it in a waterfall loop
__device__ inline __amdgpu_buffer_rsrc_t uniform_rsrc(const void* p, unsigned bytes) {
  const unsigned long long a = (unsigned long long)p;
  const unsigned long long u = ((unsigned long long)__builtin_amdgcn_readfirstlane((unsigned)(a >> 32)) << 32) |
                               (unsigned)__builtin_amdgcn_readfirstlane((unsigned)a);
  return __builtin_amdgcn_make_buffer_rsrc((void*)u, 0, (int)bytes, BUF_WORD3);
}

}  // namespace hq
