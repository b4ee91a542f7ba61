// Products with exp(s dtau K) through its Kronecker structure, for the wraps
// and the block products of the sweep.
//
// On the periodic nx x nx square lattice with nearest-neighbour hopping the
// plane-wave energies split as eps(kx, ky) = e1(kx) + e1(ky) with
// e1(k) = -2t cos k - mu/2, and the sine parts of the plane waves cancel in
// pairs k <-> -k, so exp(s dtau K) = E1 (x) E1 with E1 the nx x nx matrix
// E1[a][b] = (1/nx) sum_k cos(k (a - b)) exp(s dtau e1(k)).  With the site
// index i = ix + nx iy, (E1 (x) E1)[i][k] = E1[iy][ky] E1[ix][kx], and a
// product with it is two passes of nx-term sums per element: 4 nx n^2 flops
// in place of the 2 n^3 of a dense product (6x fewer on 12 x 12, 8x on
// 16 x 16).  At the sweep's sizes a launch is bound by the latency of one
// workgroup's load, passes and store rather than by HBM or the matrix cores.
//
// Each pass of nx-term sums is a set of small products on the matrix cores:
// for a block b of nx rows (or the nx rows b, nx + b, ...), the 16 x 16
// output D = F B with F the factor zero-padded to 16 x 16 and B 16 columns of
// the strip, by ceil(nx / 4) MFMA 16x16x4 steps.  The factor stays in each
// lane's registers as MFMA operand fragments; every strip element is read
// from LDS once per pass and written back in place (a block's reads and
// writes cover the same rows and belong to one wave).
//
// side 0 (left):  Y = diag(rs) (A (x) A) diag(ks) X diag(cs), or a chain of
//   such products with a row scale after each (a block product
//   B_{s-1} ... B_0 = diag(v_{s-1}) E ... diag(v_0) E applied to X), or
//   before each (the transposed product E diag(v_0) ... E diag(v_{s-1}) X,
//   scales taken in descending order).  One
//   workgroup per strip of KW = 16 columns of one matrix, held in LDS through
//   every step of a chain; pass 1 contracts kx within each block of rows
//   ky nx .. ky nx + nx - 1, pass 2 contracts ky across blocks.
// side 1 (right): Y = diag(rs) X diag(ks) (A (x) A) diag(cs).  One workgroup
//   per strip of 16 rows; the strip is the left operand of the products (its
//   rows the MFMA's M dimension) and the factor the right one.
//
// Strips are loaded and stored with consecutive threads on consecutive
// elements of a row.  Workgroups are mapped XCD-aware, so the left and the
// right pass over one matrix run on the same XCD and the intermediate is read
// back from that XCD's L2.  Kernels are instantiated for each nx (1 .. 16).
#include "hq_device.h"
#include "hq_internal.h"

namespace hq {

namespace {

constexpr int KW = 16;          // strip width: columns (side 0) or rows (side 1)
constexpr int KPAD = 16;        // LDS skew between consecutive blocks of nx rows (side 0)

template <int NX> struct KronDim {
  static constexpr int N = NX * NX;
  static constexpr int KS = (NX + 3) / 4;                 // MFMA k-steps per product
  static constexpr int SN = N * KW + NX * KPAD;           // side-0 strip in LDS
  static constexpr int LDR = N + 1;                       // side-1 strip row length
};

// side-0 strip element (row r, column c), rows of one block of nx skewed
template <int NX>
__device__ inline int lidx(int r, int c) { return r * KW + c + (r / NX) * KPAD; }

// LDS of the left kernel after the strip: ks, cs and the row scales of every step
template <typename T, int NX>
size_t left_lds_bytes(int steps) {
  return (size_t)KronDim<NX>::SN * sizeof(T) + (size_t)(KronDim<NX>::N + KW + steps * KronDim<NX>::N) * sizeof(double);
}

template <typename T, int NX>
__global__ __launch_bounds__(256) void kron_left_kernel(KronArgs<T> a) {
  typedef KronDim<NX> D;
  constexpr int N = D::N, KS = D::KS;
  extern __shared__ __align__(16) unsigned char kron_lds[];
  T* S = (T*)kron_lds;
  double* ksv = (double*)(S + D::SN);
  double* csv = ksv + N;
  double* rsv = csv + KW;
  constexpr int strips = (N + KW - 1) / KW;
  int z, strip;
  if (!xcd_tile(strips, a.batch, z, strip)) return;
  const int c0 = strip * KW;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const T* X = a.X + (long)z * a.sX;

  // the strip's elements, requested before the tables are built
  constexpr int PER = (N * KW + 255) / 256;
  T xin[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = tid + 256 * u, r = e / KW, c = e % KW;
    xin[u] = (e < N * KW && c0 + c < N) ? X[(long)r * N + c0 + c] : T(0);
  }
  // factor fragments: lane holds A[li][4 kk + lk] (zero outside nx x nx)
  T af[KS];
#pragma unroll
  for (int kk = 0; kk < KS; ++kk) {
    const int k = 4 * kk + lk;
    af[kk] = (li < NX && k < NX) ? a.A[li * NX + k] : T(0);
  }
  for (int i = tid; i < N; i += 256) ksv[i] = scale_value(a.ks, z, a.inner_count, i);
  if (tid < KW) csv[tid] = (c0 + tid < N) ? scale_value(a.cs, z, a.inner_count, c0 + tid) : 0.0;
  const int steps = a.steps;
  for (int e = tid; e < steps * N; e += 256) {
    const int t = e / N, i = e - t * N;
    Scale sc = a.rs;
    sc.off += (long)t * a.rstep;
    rsv[e] = scale_value(sc, z, a.inner_count, i);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = tid + 256 * u, r = e / KW, c = e % KW;
    if (e < N * KW) S[lidx<NX>(r, c)] = xin[u] * (T)ksv[r];
  }
  __syncthreads();

  const bool pre = a.pre != 0;
  for (int t = 0; t < steps; ++t) {
    const double* rt = rsv + t * N;
    // pass 1: within block b, D[ix][c] = sum_kx A[ix][kx] S[b nx + kx][c]
    // (rows scaled first in the pre-scaled form)
    for (int b = wave; b < NX; b += 4) {
      typename Frag<T>::type acc = {0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) {
        const int k = 4 * kk + lk;
        const int row = b * NX + min(k, NX - 1);
        T bv = S[lidx<NX>(row, li)];
        if (pre) bv *= (T)rt[row];
        acc = mfma16(af[kk], k < NX ? bv : T(0), acc);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = frag_row<T>(lane, v);
        if (m < NX) S[lidx<NX>(b * NX + m, li)] = acc[v];
      }
    }
    __syncthreads();
    // pass 2: for ix = b, D[iy][c] = sum_ky A[iy][ky] S[ky nx + b][c], rows
    // scaled after (the post-scaled form)
    for (int b = wave; b < NX; b += 4) {
      typename Frag<T>::type acc = {0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) {
        const int k = 4 * kk + lk;
        const T bv = S[lidx<NX>(min(k, NX - 1) * NX + b, li)];
        acc = mfma16(af[kk], k < NX ? bv : T(0), acc);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = frag_row<T>(lane, v);
        if (m < NX) {
          const int r = m * NX + b;
          S[lidx<NX>(r, li)] = pre ? acc[v] : acc[v] * (T)rt[r];
        }
      }
    }
    __syncthreads();
  }

  T* Y = a.Y + (long)z * a.sY;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = tid + 256 * u, r = e / KW, c = e % KW;
    if (e < N * KW && c0 + c < N) Y[(long)r * N + c0 + c] = S[lidx<NX>(r, c)] * (T)csv[c];
  }
}

template <typename T, int NX>
__global__ __launch_bounds__(256) void kron_right_kernel(KronArgs<T> a) {
  typedef KronDim<NX> D;
  constexpr int N = D::N, KS = D::KS, LDR = D::LDR;
  __shared__ T S[KW * LDR];
  __shared__ double rsv[KW], ksv[N], csv[N];
  constexpr int strips = (N + KW - 1) / KW;
  int z, strip;
  if (!xcd_tile(strips, a.batch, z, strip)) return;
  const int r0 = strip * KW;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const T* X = a.X + (long)z * a.sX;

  // rows r0 .. r0 + 15 are contiguous in memory
  constexpr int PER = (N * KW + 255) / 256;
  T xin[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = tid + 256 * u, r = e / N;
    xin[u] = (e < N * KW && r0 + r < N) ? X[(long)r0 * N + e] : T(0);
  }
  // factor fragments: lane holds A[4 kk + lk][li] (zero outside nx x nx)
  T bf[KS];
#pragma unroll
  for (int kk = 0; kk < KS; ++kk) {
    const int k = 4 * kk + lk;
    bf[kk] = (li < NX && k < NX) ? a.A[k * NX + li] : T(0);
  }
  for (int i = tid; i < N; i += 256) {
    ksv[i] = scale_value(a.ks, z, a.inner_count, i);
    csv[i] = scale_value(a.cs, z, a.inner_count, i);
  }
  if (tid < KW) rsv[tid] = (r0 + tid < N) ? scale_value(a.rs, z, a.inner_count, r0 + tid) : 0.0;
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = tid + 256 * u, r = e / N, c = e - r * N;
    if (e < N * KW) S[r * LDR + c] = xin[u] * (T)ksv[c];
  }
  __syncthreads();

  // pass 1: within column block b, D[r][jx] = sum_kx S[r][b nx + kx] A[kx][jx]
  for (int b = wave; b < NX; b += 4) {
    typename Frag<T>::type acc = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      const int k = 4 * kk + lk;
      const T av = S[li * LDR + b * NX + min(k, NX - 1)];
      acc = mfma16(k < NX ? av : T(0), bf[kk], acc);
    }
    if (li < NX) {
#pragma unroll
      for (int v = 0; v < 4; ++v) S[frag_row<T>(lane, v) * LDR + b * NX + li] = acc[v];
    }
  }
  __syncthreads();
  // pass 2: for jx = b, D[r][jy] = sum_ky S[r][ky nx + b] A[ky][jy]
  for (int b = wave; b < NX; b += 4) {
    typename Frag<T>::type acc = {0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      const int k = 4 * kk + lk;
      const T av = S[li * LDR + min(k, NX - 1) * NX + b];
      acc = mfma16(k < NX ? av : T(0), bf[kk], acc);
    }
    if (li < NX) {
#pragma unroll
      for (int v = 0; v < 4; ++v) S[frag_row<T>(lane, v) * LDR + li * NX + b] = acc[v];
    }
  }
  __syncthreads();

  T* Y = a.Y + (long)z * a.sY;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = tid + 256 * u, r = e / N, c = e - r * N;
    if (e < N * KW && r0 + r < N) Y[(long)r0 * N + e] = S[r * LDR + c] * (T)(rsv[r] * csv[c]);
  }
}

// A whole wrap in one launch with the matrix resident in LDS (N <= 144 in
// FP32, N <= 100 in FP64): Y = diag(rs2) (A1 (x) A1) diag(ks1) X diag(cs1)
// (A2 (x) A2) diag(cs2), one workgroup of 16 waves per matrix.  The four
// passes (kx and ky of the left product, then of the right one) run over
// units of one block and one 16-wide tile of the other index, dealt to the
// waves in turn, two units at a time; each unit reads and writes its own
// elements only.  The LDS row length is 4 mod 16, so the four 16-lane groups
// of an MFMA result (rows 4 apart) write to disjoint banks.
template <int N>
struct WrapLd { static constexpr int value = N + (20 - N % 16) % 16; };

// one unit of a pass: D = F B (left passes: F the factor, B 16 columns of
// 16 - padded rows) or D = B F (right passes: B 16 rows); rd(k, x) reads the
// strip operand (k the contracted index, x the tile index of the lane), wr(m,
// x, v) stores a result
template <typename T, int KS, bool LEFT, typename Rd, typename Wr>
__device__ inline void kron_units2(int u0, int u1, const T* fa, Rd rd, Wr wr) {
  const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
  typename Frag<T>::type acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
  T b0[KS], b1[KS];
#pragma unroll
  for (int kk = 0; kk < KS; ++kk) {
    b0[kk] = rd(u0, 4 * kk + lk, li);
    if (u1 >= 0) b1[kk] = rd(u1, 4 * kk + lk, li);
  }
#pragma unroll
  for (int kk = 0; kk < KS; ++kk) {
    acc0 = LEFT ? mfma16(fa[kk], b0[kk], acc0) : mfma16(b0[kk], fa[kk], acc0);
    if (u1 >= 0) acc1 = LEFT ? mfma16(fa[kk], b1[kk], acc1) : mfma16(b1[kk], fa[kk], acc1);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    wr(u0, frag_row<T>(lane, v), li, acc0[v]);
    if (u1 >= 0) wr(u1, frag_row<T>(lane, v), li, acc1[v]);
  }
}

template <typename T, int NX>
__global__ __launch_bounds__(1024) void kron_wrap_lds_kernel(KronWrapArgs<T> w) {
  constexpr int N = NX * NX, KS = (NX + 3) / 4, LD = WrapLd<N>::value, NTL = (N + 15) / 16;
  constexpr int UNITS = NX * NTL;
  constexpr int PER = (N * N + 1023) / 1024;
  __shared__ T S[N * LD];
  __shared__ double rs[N], cs[N];
  const int z = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const T* X = w.X + (long)z * w.sX;
  T xin[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = tid + 1024 * u;
    xin[u] = e < N * N ? X[e] : T(0);
  }
  T af[KS], bf[KS];
#pragma unroll
  for (int kk = 0; kk < KS; ++kk) {
    const int k = 4 * kk + lk;
    af[kk] = (li < NX && k < NX) ? w.A1[li * NX + k] : T(0);
    bf[kk] = (li < NX && k < NX) ? w.A2[k * NX + li] : T(0);
  }
  for (int i = tid; i < N; i += 1024) {
    rs[i] = scale_value(w.ks1, z, 1, i);
    cs[i] = scale_value(w.cs1, z, 1, i);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = tid + 1024 * u, r = e / N, c = e - r * N;
    if (e < N * N) S[r * LD + c] = xin[u] * (T)(rs[r] * cs[c]);
  }
  __syncthreads();
  for (int i = tid; i < N; i += 1024) {      // the output scales, read after the last pass
    rs[i] = scale_value(w.rs2, z, 1, i);
    cs[i] = scale_value(w.cs2, z, 1, i);
  }

  // unit u: block b = u / NTL, tile t = u % NTL (16 columns for the left
  // passes, 16 rows for the right ones); out-of-range k, columns and rows
  // read as zero from clamped addresses and are not written
  auto blk = [](int u) { return u / NTL; };
  auto t16 = [](int u) { return 16 * (u - (u / NTL) * NTL); };
  // left product, pass 1: rows b nx + kx -> b nx + ix
  for (int u = wave; u < UNITS; u += 32) {
    const int u1 = u + 16 < UNITS ? u + 16 : -1;
    kron_units2<T, KS, true>(u, u1, af,
        [&](int uu, int k, int x) {
          const int c = t16(uu) + x;
          const T v = S[(blk(uu) * NX + min(k, NX - 1)) * LD + min(c, N - 1)];
          return (k < NX && c < N) ? v : T(0);
        },
        [&](int uu, int m, int x, T v) {
          const int c = t16(uu) + x;
          if (m < NX && c < N) S[(blk(uu) * NX + m) * LD + c] = v;
        });
  }
  __syncthreads();
  // left product, pass 2: rows ky nx + b -> iy nx + b
  for (int u = wave; u < UNITS; u += 32) {
    const int u1 = u + 16 < UNITS ? u + 16 : -1;
    kron_units2<T, KS, true>(u, u1, af,
        [&](int uu, int k, int x) {
          const int c = t16(uu) + x;
          const T v = S[(min(k, NX - 1) * NX + blk(uu)) * LD + min(c, N - 1)];
          return (k < NX && c < N) ? v : T(0);
        },
        [&](int uu, int m, int x, T v) {
          const int c = t16(uu) + x;
          if (m < NX && c < N) S[(m * NX + blk(uu)) * LD + c] = v;
        });
  }
  __syncthreads();
  // right product, pass 1: columns b nx + kx -> b nx + jx
  for (int u = wave; u < UNITS; u += 32) {
    const int u1 = u + 16 < UNITS ? u + 16 : -1;
    kron_units2<T, KS, false>(u, u1, bf,
        [&](int uu, int k, int x) {
          const int r = t16(uu) + x;
          const T v = S[min(r, N - 1) * LD + blk(uu) * NX + min(k, NX - 1)];
          return (k < NX && r < N) ? v : T(0);
        },
        [&](int uu, int m, int x, T v) {
          const int r = t16(uu) + m;
          if (x < NX && r < N) S[r * LD + blk(uu) * NX + x] = v;
        });
  }
  __syncthreads();
  // right product, pass 2: columns ky nx + b -> jy nx + b
  for (int u = wave; u < UNITS; u += 32) {
    const int u1 = u + 16 < UNITS ? u + 16 : -1;
    kron_units2<T, KS, false>(u, u1, bf,
        [&](int uu, int k, int x) {
          const int r = t16(uu) + x;
          const T v = S[min(r, N - 1) * LD + min(k, NX - 1) * NX + blk(uu)];
          return (k < NX && r < N) ? v : T(0);
        },
        [&](int uu, int m, int x, T v) {
          const int r = t16(uu) + m;
          if (x < NX && r < N) S[r * LD + x * NX + blk(uu)] = v;
        });
  }
  __syncthreads();
  T* Y = w.Y + (long)z * w.sY;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int e = tid + 1024 * u, r = e / N, c = e - r * N;
    if (e < N * N) Y[e] = S[r * LD + c] * (T)(rs[r] * cs[c]);
  }
}

template <typename T, int NX>
hipError_t launch_wrap_lds_t(const KronWrapArgs<T>& w, hipStream_t s) {
  hipLaunchKernelGGL((kron_wrap_lds_kernel<T, NX>), dim3(w.batch), dim3(1024), 0, s, w);
  return hipGetLastError();
}

template <typename T, int NX>
hipError_t launch_kron_t(const KronArgs<T>& a, int side, hipStream_t s) {
  constexpr int N = NX * NX;
  const dim3 grid(xcd_grid((N + KW - 1) / KW, a.batch));
  if (side == 0) {
    const size_t lds = left_lds_bytes<T, NX>(a.steps);
    hipLaunchKernelGGL((kron_left_kernel<T, NX>), grid, dim3(256), lds, s, a);
  } else {
    hipLaunchKernelGGL((kron_right_kernel<T, NX>), grid, dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_kron_any(const KronArgs<T>& a, int side, hipStream_t s) {
  if (a.nx < 1 || a.nx > 16 || a.n != a.nx * a.nx || a.batch < 0 || a.inner_count < 1 || (side != 0 && side != 1) ||
      !a.A || !a.X || !a.Y || a.steps < 1 || (side == 1 && a.steps != 1) || a.steps * a.n > KRON_MAX_SCALES)
    return hipErrorInvalidValue;
  if (a.batch == 0) return hipSuccess;
  switch (a.nx) {
    case 1: return launch_kron_t<T, 1>(a, side, s);
    case 2: return launch_kron_t<T, 2>(a, side, s);
    case 3: return launch_kron_t<T, 3>(a, side, s);
    case 4: return launch_kron_t<T, 4>(a, side, s);
    case 5: return launch_kron_t<T, 5>(a, side, s);
    case 6: return launch_kron_t<T, 6>(a, side, s);
    case 7: return launch_kron_t<T, 7>(a, side, s);
    case 8: return launch_kron_t<T, 8>(a, side, s);
    case 9: return launch_kron_t<T, 9>(a, side, s);
    case 10: return launch_kron_t<T, 10>(a, side, s);
    case 11: return launch_kron_t<T, 11>(a, side, s);
    case 12: return launch_kron_t<T, 12>(a, side, s);
    case 13: return launch_kron_t<T, 13>(a, side, s);
    case 14: return launch_kron_t<T, 14>(a, side, s);
    case 15: return launch_kron_t<T, 15>(a, side, s);
    default: return launch_kron_t<T, 16>(a, side, s);
  }
}

template <typename T>
hipError_t launch_wrap_lds_any(const KronWrapArgs<T>& w, hipStream_t s) {
  if (!kron_wrap_lds_supported(w.nx, sizeof(T) == 4) || w.batch < 0 || !w.A1 || !w.A2 || !w.X || !w.Y)
    return hipErrorInvalidValue;
  if (w.batch == 0) return hipSuccess;
  switch (w.nx) {
    case 1: return launch_wrap_lds_t<T, 1>(w, s);
    case 2: return launch_wrap_lds_t<T, 2>(w, s);
    case 3: return launch_wrap_lds_t<T, 3>(w, s);
    case 4: return launch_wrap_lds_t<T, 4>(w, s);
    case 5: return launch_wrap_lds_t<T, 5>(w, s);
    case 6: return launch_wrap_lds_t<T, 6>(w, s);
    case 7: return launch_wrap_lds_t<T, 7>(w, s);
    case 8: return launch_wrap_lds_t<T, 8>(w, s);
    case 9: return launch_wrap_lds_t<T, 9>(w, s);
    case 10: return launch_wrap_lds_t<T, 10>(w, s);
    default:
      if constexpr (sizeof(T) == 4) {
        if (w.nx == 11) return launch_wrap_lds_t<T, 11>(w, s);
        return launch_wrap_lds_t<T, 12>(w, s);
      }
      return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_kron(const KronArgs<double>& a, int side, hipStream_t s) { return launch_kron_any(a, side, s); }
hipError_t launch_kron(const KronArgs<float>& a, int side, hipStream_t s) { return launch_kron_any(a, side, s); }

bool kron_wrap_lds_supported(int nx, bool fp32) { return nx >= 1 && nx <= (fp32 ? 12 : 10); }
hipError_t launch_kron_wrap_lds(const KronWrapArgs<double>& w, hipStream_t s) { return launch_wrap_lds_any(w, s); }
hipError_t launch_kron_wrap_lds(const KronWrapArgs<float>& w, hipStream_t s) { return launch_wrap_lds_any(w, s); }

}  // namespace hq
