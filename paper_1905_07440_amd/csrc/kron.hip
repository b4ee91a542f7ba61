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
// 16 x 16).  Bandwidth, not arithmetic, bounds these kernels.
//
// side 0 (left):  Y = diag(rs) (A (x) A) diag(ks) X diag(cs), or a chain of
//   such products with a row scale after each (a block product
//   B_{s-1} ... B_0 = diag(v_{s-1}) E ... diag(v_0) E from X = I).  One
//   workgroup per strip of KW columns of one matrix; the strip stays in LDS
//   through every step of a chain.  Pass 1 contracts kx: a thread takes the
//   fiber (ky, column c) of nx values X[ky nx + kx][c] (the first straight
//   from memory, the 16 threads of one ky reading 16 consecutive columns) and
//   writes its nx sums back in place.  Pass 2 contracts ky: thread (ix, c)
//   reads its fiber and writes the nx outputs of rows iy nx + ix.
// side 1 (right): Y = diag(rs) X diag(ks) (A (x) A) diag(cs).  One workgroup
//   per strip of KW rows.  Pass 1 contracts kx over the contiguous runs
//   X[r][ky nx .. ky nx + nx - 1] (thread (r, ky), consecutive threads on
//   consecutive runs of a row), pass 2 contracts ky through LDS.
//
// Both are instantiated for each nx (1 .. 16), so that every loop has a
// compile-time length and no load or LDS access sits behind a branch; the
// first fibers are requested from memory before the factor and the diagonal
// scales are set up in LDS.  Workgroups are mapped XCD-aware, so the left and
// the right pass over one matrix run on the same XCD and the intermediate is
// read back from that XCD's L2.
#include "hq_device.h"
#include "hq_internal.h"

namespace hq {

namespace {

constexpr int KW = 16;          // strip width (columns, or rows for side 1)
constexpr int KPAD = 16;        // LDS skew between the fibers of consecutive ky

// LDS of the left kernel: the skewed strip, the factor, ks, cs and the row
// scales of every step
template <typename T, int NX>
struct LeftLayout {
  static constexpr int N = NX * NX;
  static constexpr int SN = N * KW + NX * KPAD;
  static constexpr int AN = (NX * NX + 1) & ~1;      // keeps the doubles 8-byte aligned
  static size_t bytes(int steps) { return (size_t)(SN + AN) * sizeof(T) + (size_t)(N + KW + steps * N) * sizeof(double); }
};

__device__ inline int sidx(int r, int j, int blk) { return r * KW + j + blk * KPAD; }

template <typename T, int NX>
__global__ __launch_bounds__(256) void kron_left_kernel(KronArgs<T> a) {
  typedef LeftLayout<T, NX> Lay;
  constexpr int N = Lay::N;
  extern __shared__ __align__(16) unsigned char kron_lds[];
  T* S = (T*)kron_lds;
  T* As = S + Lay::SN;
  double* ksv = (double*)(As + Lay::AN);
  double* csv = ksv + N;
  double* rsv = csv + KW;
  constexpr int strips = (N + KW - 1) / KW;
  int z, strip;
  if (!xcd_tile(strips, a.batch, z, strip)) return;
  const int c0 = strip * KW;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int j = tid % KW, f = tid / KW;
  const bool act = f < NX, col_ok = c0 + j < N;
  const T* X = a.X + (long)z * a.sX;
  T v[NX];
  if (act && col_ok) {
#pragma unroll
    for (int kx = 0; kx < NX; ++kx) v[kx] = X[(long)(f * NX + kx) * N + c0 + j];
  } else {
#pragma unroll
    for (int kx = 0; kx < NX; ++kx) v[kx] = T(0);
  }
  for (int e = tid; e < NX * NX; e += nt) As[e] = a.A[e];
  for (int i = tid; i < N; i += nt) ksv[i] = scale_value(a.ks, z, a.inner_count, i);
  if (tid < KW) csv[tid] = col_ok ? scale_value(a.cs, z, a.inner_count, c0 + tid) : 0.0;
  const int steps = a.steps;
  for (int e = tid; e < steps * N; e += nt) {
    const int t = e / N, i = e - t * N;
    Scale sc = a.rs;
    sc.off += (long)t * a.rstep;
    rsv[e] = scale_value(sc, z, a.inner_count, i);
  }
  __syncthreads();

  T* Y = a.Y + (long)z * a.sY;
  for (int t = 0; t < steps; ++t) {
    if (act) {                           // pass 1: fiber (ky = f, column c0 + j)
      if (t == 0) {
#pragma unroll
        for (int kx = 0; kx < NX; ++kx) v[kx] *= (T)ksv[f * NX + kx];
      } else {
#pragma unroll
        for (int kx = 0; kx < NX; ++kx) v[kx] = S[sidx(f * NX + kx, j, f)];
      }
#pragma unroll
      for (int ix = 0; ix < NX; ++ix) {
        T s = T(0);
#pragma unroll
        for (int kx = 0; kx < NX; ++kx) s = fma(As[ix * NX + kx], v[kx], s);
        S[sidx(f * NX + ix, j, f)] = s;
      }
    }
    __syncthreads();
    const bool last = t + 1 == steps;
    if (act) {                           // pass 2: fiber (ix = f, column c0 + j)
      T h[NX];
#pragma unroll
      for (int ky = 0; ky < NX; ++ky) h[ky] = S[sidx(ky * NX + f, j, ky)];
      const double* rt = rsv + t * N;
#pragma unroll
      for (int iy = 0; iy < NX; ++iy) {
        T s = T(0);
#pragma unroll
        for (int ky = 0; ky < NX; ++ky) s = fma(As[iy * NX + ky], h[ky], s);
        const int r = iy * NX + f;
        if (!last) S[sidx(r, j, iy)] = (T)rt[r] * s;
        else if (col_ok) Y[(long)r * N + c0 + j] = (T)(rt[r] * csv[j]) * s;
      }
    }
    if (!last) __syncthreads();
  }
}

template <typename T, int NX>
__global__ __launch_bounds__(256) void kron_right_kernel(KronArgs<T> a) {
  constexpr int N = NX * NX;
  constexpr int SP = N + 1;              // LDS row length
  __shared__ T S[KW * SP];
  __shared__ T As[NX * NX];
  __shared__ double rsv[KW], ksv[N], csv[N];
  constexpr int strips = (N + KW - 1) / KW;
  int z, strip;
  if (!xcd_tile(strips, a.batch, z, strip)) return;
  const int r0 = strip * KW;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int r = tid / NX, q = tid - r * NX;   // row of the strip; ky (pass 1) or jx (pass 2)
  const bool row_ok = r < KW && r0 + r < N;
  const T* X = a.X + (long)z * a.sX;
  T v[NX];
  if (row_ok) {
    const T* xr = X + (long)(r0 + r) * N + q * NX;
#pragma unroll
    for (int kx = 0; kx < NX; ++kx) v[kx] = xr[kx];
  } else {
#pragma unroll
    for (int kx = 0; kx < NX; ++kx) v[kx] = T(0);
  }
  for (int e = tid; e < NX * NX; e += nt) As[e] = a.A[e];
  for (int i = tid; i < N; i += nt) {
    ksv[i] = scale_value(a.ks, z, a.inner_count, i);
    csv[i] = scale_value(a.cs, z, a.inner_count, i);
  }
  if (tid < KW) rsv[tid] = (r0 + tid < N) ? scale_value(a.rs, z, a.inner_count, r0 + tid) : 0.0;
  __syncthreads();

  T* Y = a.Y + (long)z * a.sY;
  if (row_ok) {                          // pass 1: run (row r0 + r, ky = q)
#pragma unroll
    for (int kx = 0; kx < NX; ++kx) v[kx] *= (T)ksv[q * NX + kx];
#pragma unroll
    for (int jx = 0; jx < NX; ++jx) {
      T s = T(0);
#pragma unroll
      for (int kx = 0; kx < NX; ++kx) s = fma(v[kx], As[kx * NX + jx], s);
      S[r * SP + q * NX + jx] = s;
    }
  }
  __syncthreads();
  if (row_ok) {                          // pass 2: fiber (row r0 + r, jx = q)
    T h[NX];
#pragma unroll
    for (int ky = 0; ky < NX; ++ky) h[ky] = S[r * SP + ky * NX + q];
    const double ri = rsv[r];
    T* yr = Y + (long)(r0 + r) * N + q;
#pragma unroll
    for (int jy = 0; jy < NX; ++jy) {
      T s = T(0);
#pragma unroll
      for (int ky = 0; ky < NX; ++ky) s = fma(h[ky], As[ky * NX + jy], s);
      yr[jy * NX] = (T)(ri * csv[jy * NX + q]) * s;
    }
  }
}

template <typename T, int NX>
hipError_t launch_kron_t(const KronArgs<T>& a, int side, hipStream_t s) {
  constexpr int N = NX * NX;
  const unsigned threads = (unsigned)(64 * ((NX * KW + 63) / 64));
  const dim3 grid(xcd_grid((N + KW - 1) / KW, a.batch));
  if (side == 0) {
    const size_t lds = LeftLayout<T, NX>::bytes(a.steps);
    hipLaunchKernelGGL((kron_left_kernel<T, NX>), grid, dim3(threads), lds, s, a);
  } else {
    hipLaunchKernelGGL((kron_right_kernel<T, NX>), grid, dim3(threads), 0, s, a);
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

}  // namespace

hipError_t launch_kron(const KronArgs<double>& a, int side, hipStream_t s) { return launch_kron_any(a, side, s); }
hipError_t launch_kron(const KronArgs<float>& a, int side, hipStream_t s) { return launch_kron_any(a, side, s); }

}  // namespace hq
