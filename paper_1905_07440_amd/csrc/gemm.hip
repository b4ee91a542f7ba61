// Batched dense products on MFMA for the UDT combines and merges of the DQMC
// sweep, the pairwise merges of a from-scratch recompute, and the dense wrap
// forms (the products with exp(dtau K) otherwise take its Kronecker form).  C = alpha * diag(rs) op(A) diag(ks) op(B)
// diag(cs) + beta * C, row-major, one workgroup per (tile, batch entry).
//
// FP64 uses v_mfma_f64_16x16x4f64, FP32 uses v_mfma_f32_16x16x4f32 with
// FP32 accumulation.  A workgroup tile of BM x BN is split over WM x WN
// waves, each computing FM x FN fragments of 16 x 16; K advances in stages
// of BK = 16 through two LDS buffers, the next stage's loads in flight while
// the current one is multiplied.  Edges are zero-padded on load and masked
// on store, so any M, N, K works.
#include "hq_device.h"
#include "hq_internal.h"

namespace hq {

// K staged 16 at a time through two LDS buffers: while the waves multiply
// out of one buffer, every thread's loads of the next 16-wide K chunk are in
// flight, and one barrier per chunk separates the two.  Loads and stores go
// through buffer resources with masked byte offsets: a thread's offsets into
// op(A) and op(B) are set once (rows past M or N already outside) and step by
// one chunk's stride, an index past K takes the outside offset, so the loop
// has no per-element bounds branches and no 64-bit address arithmetic.
template <typename T, int BM, int BN, int WM, int WN, bool TA, bool TB>
__device__ __forceinline__ void gemm_tile(const GemmArgs<T>& a, int z, int tile) {
  constexpr int NT = WM * WN * 64;
  constexpr int BK = 16;
  constexpr int FM = BM / (WM * 16), FN = BN / (WN * 16);
  constexpr int PA = (BM * BK + NT - 1) / NT, PB = (BN * BK + NT - 1) / NT;   // loads per thread per chunk
  constexpr int PAD = 1;
  constexpr unsigned ES = sizeof(T);
  static_assert(FM >= 1 && FN >= 1, "tile too small");
  __shared__ T As[2][BK][BM + PAD];
  __shared__ T Bs[2][BK][BN + PAD];
  __shared__ double rsv[BM];
  __shared__ double csv[BN];
  __shared__ double ksv[256 + 16];   // K <= 256, plus the zero chunk after the last

  const int tn = (a.N + BN - 1) / BN;
  const int m0 = (tile / tn) * BM, n0 = (tile % tn) * BN;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WN, wn = wave % WN;
  // resources over this batch entry's storage of A (M x K, or K x M when
  // transposed), B and C; every in-range element lies inside them
  const __amdgpu_buffer_rsrc_t ra_ = uniform_rsrc(a.A + batch_offset(z, a.split, a.sA, a.sAo),
                                                  (unsigned)((TA ? a.K : a.M) * a.lda) * ES);
  const __amdgpu_buffer_rsrc_t rb_ = uniform_rsrc(a.B + batch_offset(z, a.split, a.sB, a.sBo),
                                                  (unsigned)((TB ? a.N : a.K) * a.ldb) * ES);
  const __amdgpu_buffer_rsrc_t rc_ = uniform_rsrc(a.C + batch_offset(z, a.split, a.sC, a.sCo),
                                                  (unsigned)(a.M * a.ldc) * ES);
  const int nchunk = (a.K + BK - 1) / BK;

  for (int i = tid; i < BM; i += NT)
    rsv[i] = (m0 + i < a.M) ? scale_value(a.rs, z, a.inner_count, m0 + i) : 0.0;
  for (int i = tid; i < BN; i += NT)
    csv[i] = (n0 + i < a.N) ? scale_value(a.cs, z, a.inner_count, n0 + i) : 0.0;
  // the inner scale (1 without one; 0 from K to the end of the chunk after
  // the last, where rb is 0 as well): every B element is scaled on its way
  // into LDS, with no test
  for (int i = tid; i < BK * (nchunk + 1); i += NT) ksv[i] = (i < a.K) ? scale_value(a.ks, z, a.inner_count, i) : 0.0;

  // chunk element e -> (row, k), consecutive threads on the source's
  // contiguous index; per load: byte offset at chunk 0, k within the chunk,
  // LDS slot (-1: past the chunk, when NT does not divide it)
  unsigned oa[PA], ob[PB];
  int ka[PA], kb[PB], sa[PA], sb[PB];
#pragma unroll
  for (int q = 0; q < PA; ++q) {
    const int e = tid + NT * q;
    const int m = TA ? e % BM : e / BK, k = TA ? e / BM : e % BK;
    const bool live = e < BM * BK && m0 + m < a.M;
    oa[q] = live ? (unsigned)(TA ? k * a.lda + m0 + m : (m0 + m) * a.lda + k) * ES : BUF_OUTSIDE;
    ka[q] = k;
    sa[q] = (e < BM * BK) ? k * (BM + PAD) + m : -1;
  }
#pragma unroll
  for (int q = 0; q < PB; ++q) {
    const int e = tid + NT * q;
    const int n = TB ? e / BK : e % BN, k = TB ? e % BK : e / BN;
    const bool live = e < BN * BK && n0 + n < a.N;
    ob[q] = live ? (unsigned)(TB ? (n0 + n) * a.ldb + k : k * a.ldb + n0 + n) * ES : BUF_OUTSIDE;
    kb[q] = k;
    sb[q] = (e < BN * BK) ? k * (BN + PAD) + n : -1;
  }
  const unsigned stepA = (unsigned)(TA ? BK * a.lda : BK) * ES;   // one chunk further along K
  const unsigned stepB = (unsigned)(TB ? BK : BK * a.ldb) * ES;

  // two register sets: the loads of chunk c + 2 go out while chunk c is
  // multiplied, so each load has two chunks' work to arrive in.  Loads and
  // stores take no branches (a chunk past K reads zeros through the outside
  // offset), so the wait before a store covers only the set it stores.
  T ra[2][PA], rb[2][PB];
  auto load = [&](int c, int set) {
    const int kc = BK * c;
#pragma unroll
    for (int q = 0; q < PA; ++q)
      ra[set][q] = buf_load(ra_, (kc + ka[q] < a.K) ? oa[q] + c * stepA : BUF_OUTSIDE, (T*)nullptr);
#pragma unroll
    for (int q = 0; q < PB; ++q)
      rb[set][q] = buf_load(rb_, (kc + kb[q] < a.K) ? ob[q] + c * stepB : BUF_OUTSIDE, (T*)nullptr);
  };
  auto store = [&](int c, int set, int buf) {
#pragma unroll
    for (int q = 0; q < PA; ++q)
      if (PA * NT == BM * BK || sa[q] >= 0) (&As[buf][0][0])[sa[q]] = ra[set][q];
#pragma unroll
    for (int q = 0; q < PB; ++q)
      if (PB * NT == BN * BK || sb[q] >= 0) (&Bs[buf][0][0])[sb[q]] = (T)((double)rb[set][q] * ksv[BK * c + kb[q]]);
  };

  typedef typename Frag<T>::type F;
  F acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = F{0, 0, 0, 0};
  auto multiply = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T af[FM], bf[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) af[i] = As[buf][kk + (lane >> 4)][wm * FM * 16 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < FN; ++j) bf[j] = Bs[buf][kk + (lane >> 4)][wn * FN * 16 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = mfma16(af[i], bf[j], acc[i][j]);
    }
  };

  load(0, 0);
  load(1, 1);
  __syncthreads();                         // rsv, csv, ksv
  store(0, 0, 0);
  __syncthreads();
  // chunk c sits in LDS buffer c & 1 and came through register set c & 1;
  // a pair of chunks per trip keeps the set and buffer indices static
  int c = 0;
  for (; c + 1 < nchunk; c += 2) {
    load(c + 2, 0);
    multiply(0);
    store(c + 1, 1, 1);                    // buffer 1 was last read before the previous barrier
    __syncthreads();
    load(c + 3, 1);
    multiply(1);
    store(c + 2, 0, 0);                    // zeros when c + 2 = nchunk
    __syncthreads();
  }
  if (c < nchunk) multiply(0);             // an odd last chunk, in buffer 0

  // C through the resource: elements past M or N take the outside offset
  // (the beta read gives 0 there and the store is dropped)
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int lr = wm * FM * 16 + i * 16 + frag_row<T>(lane, v);
        const int lc = wn * FN * 16 + j * 16 + (lane & 15);
        const int r = m0 + lr, c = n0 + lc;
        const unsigned off = (r < a.M && c < a.N) ? (unsigned)(r * a.ldc + c) * ES : BUF_OUTSIDE;
        double val = a.alpha * rsv[lr] * (double)acc[i][j][v] * csv[lc];
        if (a.beta != 0.0) val += a.beta * (double)buf_load(rc_, off, (T*)nullptr);
        buf_store((T)val, rc_, off);
      }
}

// TA, TB: the transposition flags of a, fixed per instantiation
template <typename T, int BM, int BN, int WM, int WN, bool TA, bool TB>
__global__ __launch_bounds__(WM * WN * 64) void gemm_kernel(GemmArgs<T> a) {
  int z, tile;
  if (!xcd_tile(((a.N + BN - 1) / BN) * ((a.M + BM - 1) / BM), a.batch, z, tile)) return;
  gemm_tile<T, BM, BN, WM, WN, TA, TB>(a, z, tile);
}

// two independent products of one shape and the same transpositions in one
// launch: batch entries [0, a.batch) are a's, the next b.batch are b's
template <typename T, int BM, int BN, int WM, int WN, bool TA, bool TB>
__global__ __launch_bounds__(WM * WN * 64) void gemm_pair_kernel(GemmArgs<T> a, GemmArgs<T> b) {
  int z, tile;
  if (!xcd_tile(((a.N + BN - 1) / BN) * ((a.M + BM - 1) / BM), a.batch + b.batch, z, tile)) return;
  if (z < a.batch)
    gemm_tile<T, BM, BN, WM, WN, TA, TB>(a, z, tile);
  else
    gemm_tile<T, BM, BN, WM, WN, TA, TB>(b, z - a.batch, tile);
}

// Direct-load variant: the operands do not pass through LDS.  Each wave owns
// a (16 FM) x (16 FN) block of C and fetches its own MFMA operands straight
// into registers, one 16-wide K chunk ahead of the MFMAs that use them.  The
// chunk's k are spread over the four lane groups so that lane (r, g), r =
// lane & 15, g = lane >> 4, holds k = 16 c + 4 g + s (s = 0 .. 3) of row r of
// each of its A blocks and of column r of each of its B blocks, and MFMA
// step s sums over those four k (a relabelling of k within the chunk, the
// same on both operands).  No barrier sits inside the K loop: the W waves of
// a workgroup (stacked over rows, sharing the B columns, whose loads then
// meet in the L1 cache) run independently.  Masked buffer offsets zero
// everything past M, N or K.
template <typename T, int FM, int FN, int W, bool TA, bool TB>
__global__ __launch_bounds__(W * 64) void gemm_direct_kernel(GemmArgs<T> a) {
  constexpr int BM = 16 * FM * W, BN = 16 * FN, NT = W * 64;
  constexpr unsigned ES = sizeof(T);
  __shared__ double rsv[BM];
  __shared__ double csv[BN];
  __shared__ double ksv[256 + 16];         // K <= 256, plus the zero chunk after the last

  const int tn = (a.N + BN - 1) / BN, tm = (a.M + BM - 1) / BM;
  int z, tile;
  if (!xcd_tile(tn * tm, a.batch, z, tile)) return;
  const int m0 = (tile / tn) * BM, n0 = (tile % tn) * BN;
  const int tid = threadIdx.x, lane = tid & 63, r = lane & 15, g = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nchunk = (a.K + 15) / 16;
  const __amdgpu_buffer_rsrc_t ra_ = uniform_rsrc(a.A + batch_offset(z, a.split, a.sA, a.sAo),
                                                  (unsigned)((TA ? a.K : a.M) * a.lda) * ES);
  const __amdgpu_buffer_rsrc_t rb_ = uniform_rsrc(a.B + batch_offset(z, a.split, a.sB, a.sBo),
                                                  (unsigned)((TB ? a.N : a.K) * a.ldb) * ES);
  const __amdgpu_buffer_rsrc_t rc_ = uniform_rsrc(a.C + batch_offset(z, a.split, a.sC, a.sCo),
                                                  (unsigned)(a.M * a.ldc) * ES);

  for (int i = tid; i < BM; i += NT)
    rsv[i] = (m0 + i < a.M) ? scale_value(a.rs, z, a.inner_count, m0 + i) : 0.0;
  for (int i = tid; i < BN; i += NT)
    csv[i] = (n0 + i < a.N) ? scale_value(a.cs, z, a.inner_count, n0 + i) : 0.0;
  const bool kscale = a.ks.v != nullptr;
  if (kscale)
    for (int i = tid; i < 16 * nchunk; i += NT) ksv[i] = (i < a.K) ? scale_value(a.ks, z, a.inner_count, i) : 0.0;
  __syncthreads();

  // byte offsets of this lane's elements at chunk 0, s = 0 (outside past M or N)
  const int wr0 = m0 + wave * 16 * FM;
  unsigned oa[FM], ob[FN];
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    const int row = wr0 + 16 * i + r;
    oa[i] = (row < a.M) ? (unsigned)(TA ? 4 * g * a.lda + row : row * a.lda + 4 * g) * ES : BUF_OUTSIDE;
  }
#pragma unroll
  for (int j = 0; j < FN; ++j) {
    const int col = n0 + 16 * j + r;
    ob[j] = (col < a.N) ? (unsigned)(TB ? col * a.ldb + 4 * g : 4 * g * a.ldb + col) * ES : BUF_OUTSIDE;
  }
  const unsigned sA = (unsigned)(TA ? a.lda : 1) * ES, sB = (unsigned)(TB ? 1 : a.ldb) * ES;   // k + 1
  const unsigned cA = 16 * sA, cB = 16 * sB;                                                    // chunk + 1

  T va[2][FM][4], vb[2][FN][4];
  auto load = [&](int c, int set) {
    const int kg = 16 * c + 4 * g;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      // bit 31 (past every resource) when k = kg + t >= K: arithmetic, not a
      // select, which the compiler would turn into a branch around the load
      const unsigned out = (unsigned)(a.K - 1 - kg - t) & BUF_OUTSIDE;
#pragma unroll
      for (int i = 0; i < FM; ++i) va[set][i][t] = buf_load(ra_, (oa[i] + c * cA + t * sA) | out, (T*)nullptr);
#pragma unroll
      for (int j = 0; j < FN; ++j) vb[set][j][t] = buf_load(rb_, (ob[j] + c * cB + t * sB) | out, (T*)nullptr);
    }
  };
  typedef typename Frag<T>::type F;
  F acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = F{0, 0, 0, 0};
  auto multiply = [&](int c, int set) {
    if (kscale) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double kv = ksv[16 * c + 4 * g + t];
#pragma unroll
        for (int j = 0; j < FN; ++j) vb[set][j][t] = (T)((double)vb[set][j][t] * kv);
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = mfma16(va[set][i][t], vb[set][j][t], acc[i][j]);
  };

  // chunk c comes through register set c & 1; loads of chunk c + 1 are in
  // flight while chunk c is multiplied (a chunk past K loads zeros)
  load(0, 0);
  int c = 0;
  for (; c + 1 < nchunk; c += 2) {
    load(c + 1, 1);
    multiply(c, 0);
    load(c + 2, 0);
    multiply(c + 1, 1);
  }
  if (c < nchunk) multiply(c, 0);

#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int lr = wave * 16 * FM + i * 16 + frag_row<T>(lane, v);
        const int lc = j * 16 + r;
        const int row = m0 + lr, col = n0 + lc;
        const unsigned off = (row < a.M && col < a.N) ? (unsigned)(row * a.ldc + col) * ES : BUF_OUTSIDE;
        double val = a.alpha * rsv[lr] * (double)acc[i][j][v] * csv[lc];
        if (a.beta != 0.0) val += a.beta * (double)buf_load(rc_, off, (T*)nullptr);
        buf_store((T)val, rc_, off);
      }
}

// Full-K variant for K <= a few hundred (every DQMC product has K = N <= 256):
// the whole BM x K panel of op(A) and K x BN panel of op(B) are staged in LDS
// in one pass, so a tile pays the memory latency once instead of once per K
// stage.  LDS: (BM + BN + 2) * K elements, dynamic.
template <typename T, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(WM * WN * 64) void gemm_fullk_kernel(GemmArgs<T> a) {
  constexpr int NT = WM * WN * 64;
  constexpr int FM = BM / (WM * 16), FN = BN / (WN * 16);
  constexpr int LA = BM + 1, LB = BN + 1;  // odd strides: the transposing stores hit distinct banks
  static_assert(FM >= 1 && FN >= 1, "tile too small");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* As = (T*)smem_raw;                    // [K4][LA]: As[k][m] = op(A)(m0 + m, k)
  const int K4 = (a.K + 3) & ~3;
  T* Bs = As + (long)K4 * LA;              // [K4][LB]: Bs[k][n] = op(B)(k, n0 + n)
  __shared__ double rsv[BM];
  __shared__ double csv[BN];
  __shared__ double ksv[256];

  const int tn = (a.N + BN - 1) / BN, tm = (a.M + BM - 1) / BM;
  int z, tile;
  if (!xcd_tile(tn * tm, a.batch, z, tile)) return;
  const int m0 = (tile / tn) * BM, n0 = (tile % tn) * BN;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WN, wn = wave % WN;
  const T* A = a.A + batch_offset(z, a.split, a.sA, a.sAo);
  const T* B = a.B + batch_offset(z, a.split, a.sB, a.sBo);
  T* C = a.C + batch_offset(z, a.split, a.sC, a.sCo);

  for (int i = tid; i < BM; i += NT)
    rsv[i] = (m0 + i < a.M) ? scale_value(a.rs, z, a.inner_count, m0 + i) : 0.0;
  for (int i = tid; i < BN; i += NT)
    csv[i] = (n0 + i < a.N) ? scale_value(a.cs, z, a.inner_count, n0 + i) : 0.0;
  const bool kscale = a.ks.v != nullptr;
  if (kscale)
    for (int i = tid; i < a.K; i += NT) ksv[i] = scale_value(a.ks, z, a.inner_count, i);
  __syncthreads();
  // op(A) and op(B) panels, 16 consecutive threads along the contiguous
  // index of the source (coalesced), no per-element division
  {
    const int t16 = tid & 15, g16 = tid >> 4;
    constexpr int G = NT / 16;             // thread groups of 16
    if (!a.tA) {                           // A[m][k]: groups over m, lanes over k
      for (int m = g16; m < BM; m += G) {
        const int gm = m0 + m;
#pragma unroll 4
        for (int k = t16; k < K4; k += 16)
          As[k * LA + m] = (gm < a.M && k < a.K) ? A[(long)gm * a.lda + k] : T(0);
      }
    } else {                               // A[k][m]: groups over k, lanes over m
      for (int k = g16; k < K4; k += G)
#pragma unroll
        for (int m = t16; m < BM; m += 16) {
          const int gm = m0 + m;
          As[k * LA + m] = (gm < a.M && k < a.K) ? A[(long)k * a.lda + gm] : T(0);
        }
    }
    if (!a.tB) {                           // B[k][n]: groups over k, lanes over n
      for (int k = g16; k < K4; k += G)
#pragma unroll
        for (int n = t16; n < BN; n += 16) {
          const int gn = n0 + n;
          Bs[k * LB + n] = (gn < a.N && k < a.K) ? (T)((double)B[(long)k * a.ldb + gn] * (kscale ? ksv[k] : 1.0))
                                                 : T(0);
        }
    } else {                               // B[n][k]: groups over n, lanes over k
      for (int n = g16; n < BN; n += G) {
        const int gn = n0 + n;
#pragma unroll 4
        for (int k = t16; k < K4; k += 16)
          Bs[k * LB + n] = (gn < a.N && k < a.K) ? (T)((double)B[(long)gn * a.ldb + k] * (kscale ? ksv[k] : 1.0))
                                                 : T(0);
      }
    }
  }
  __syncthreads();

  typedef typename Frag<T>::type F;
  F acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = F{0, 0, 0, 0};
  for (int kk = 0; kk < K4; kk += 4) {
    T af[FM], bf[FN];
#pragma unroll
    for (int i = 0; i < FM; ++i) af[i] = As[(kk + (lane >> 4)) * LA + wm * FM * 16 + i * 16 + (lane & 15)];
#pragma unroll
    for (int j = 0; j < FN; ++j) bf[j] = Bs[(kk + (lane >> 4)) * LB + wn * FN * 16 + j * 16 + (lane & 15)];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] = mfma16(af[i], bf[j], acc[i][j]);
  }

#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int lr = wm * FM * 16 + i * 16 + frag_row<T>(lane, v);
        const int lc = wn * FN * 16 + j * 16 + (lane & 15);
        const int r = m0 + lr, c = n0 + lc;
        if (r < a.M && c < a.N) {
          double val = a.alpha * rsv[lr] * (double)acc[i][j][v] * csv[lc];
          T* dst = C + (long)r * a.ldc + c;
          if (a.beta != 0.0) val += a.beta * (double)(*dst);
          *dst = (T)val;
        }
      }
}

// Register-prefetch variant: every thread loads its share of the whole
// BM x K panel of op(A) and K x BN panel of op(B) into registers at once (one
// memory latency for the tile), then the K extent passes through two small
// LDS buffers 16 at a time.  LDS stays small, so many tiles share a CU.
// KC = number of 16-wide K chunks the registers can hold (K <= 16 KC).
template <typename T, int BM, int BN, int WM, int WN, int KC>
__global__ __launch_bounds__(WM * WN * 64) void gemm_regpf_kernel(GemmArgs<T> a) {
  constexpr int NT = WM * WN * 64;
  constexpr int BK = 16;
  constexpr int FM = BM / (WM * 16), FN = BN / (WN * 16);
  constexpr int PA = BM * BK / NT, PB = BN * BK / NT;   // elements per thread per chunk
  static_assert(PA * NT == BM * BK && PB * NT == BN * BK, "tile must split evenly");
  constexpr int PAD = 1;
  __shared__ T As[2][BK][BM + PAD];
  __shared__ T Bs[2][BK][BN + PAD];
  __shared__ double rsv[BM];
  __shared__ double csv[BN];
  __shared__ double ksv[256];

  const int tn = (a.N + BN - 1) / BN, tm = (a.M + BM - 1) / BM;
  int z, tile;
  if (!xcd_tile(tn * tm, a.batch, z, tile)) return;
  const int m0 = (tile / tn) * BM, n0 = (tile % tn) * BN;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave / WN, wn = wave % WN;
  const T* A = a.A + batch_offset(z, a.split, a.sA, a.sAo);
  const T* B = a.B + batch_offset(z, a.split, a.sB, a.sBo);
  T* C = a.C + batch_offset(z, a.split, a.sC, a.sCo);
  const int nchunk = (a.K + BK - 1) / BK;

  for (int i = tid; i < BM; i += NT)
    rsv[i] = (m0 + i < a.M) ? scale_value(a.rs, z, a.inner_count, m0 + i) : 0.0;
  for (int i = tid; i < BN; i += NT)
    csv[i] = (n0 + i < a.N) ? scale_value(a.cs, z, a.inner_count, n0 + i) : 0.0;
  const bool kscale = a.ks.v != nullptr;
  if (kscale)
    for (int i = tid; i < a.K; i += NT) ksv[i] = scale_value(a.ks, z, a.inner_count, i);

  // element e of a chunk -> (row, k) with consecutive threads on the source's contiguous index
  auto a_pos = [&](int e, int& m, int& k) {
    if (a.tA) { m = e % BM; k = e / BM; } else { m = e / BK; k = e % BK; }
  };
  auto b_pos = [&](int e, int& k, int& n) {
    if (a.tB) { n = e / BK; k = e % BK; } else { k = e / BN; n = e % BN; }
  };
  T ra[KC][PA], rb[KC][PB];
#pragma unroll
  for (int c = 0; c < KC; ++c) {
#pragma unroll
    for (int q = 0; q < PA; ++q) {
      int m, k;
      a_pos(tid + NT * q, m, k);
      const int gm = m0 + m, gk = BK * c + k;
      ra[c][q] = (c < nchunk && gm < a.M && gk < a.K) ? (a.tA ? A[(long)gk * a.lda + gm] : A[(long)gm * a.lda + gk])
                                                      : T(0);
    }
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      int k, n;
      b_pos(tid + NT * q, k, n);
      const int gn = n0 + n, gk = BK * c + k;
      rb[c][q] = (c < nchunk && gn < a.N && gk < a.K) ? (a.tB ? B[(long)gn * a.ldb + gk] : B[(long)gk * a.ldb + gn])
                                                      : T(0);
    }
  }
  __syncthreads();                         // rsv, csv, ksv

  typedef typename Frag<T>::type F;
  F acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = F{0, 0, 0, 0};
#pragma unroll
  for (int c = 0; c < KC; ++c) {
    if (c < nchunk) {                      // the same for every thread
      const int buf = c & 1;
#pragma unroll
      for (int q = 0; q < PA; ++q) {
        int m, k;
        a_pos(tid + NT * q, m, k);
        As[buf][k][m] = ra[c][q];
      }
#pragma unroll
      for (int q = 0; q < PB; ++q) {
        int k, n;
        b_pos(tid + NT * q, k, n);
        const int gk = BK * c + k;        // rb is 0 past K; ksv is only written below K
        Bs[buf][k][n] = (kscale && gk < a.K) ? (T)((double)rb[c][q] * ksv[gk]) : rb[c][q];
      }
      __syncthreads();                     // buffer c & 1 is complete; buffer (c+1) & 1 was read before the last barrier
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        T af[FM], bf[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) af[i] = As[buf][kk + (lane >> 4)][wm * FM * 16 + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < FN; ++j) bf[j] = Bs[buf][kk + (lane >> 4)][wn * FN * 16 + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) acc[i][j] = mfma16(af[i], bf[j], acc[i][j]);
      }
    }
  }

#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int lr = wm * FM * 16 + i * 16 + frag_row<T>(lane, v);
        const int lc = wn * FN * 16 + j * 16 + (lane & 15);
        const int r = m0 + lr, c = n0 + lc;
        if (r < a.M && c < a.N) {
          double val = a.alpha * rsv[lr] * (double)acc[i][j][v] * csv[lc];
          T* dst = C + (long)r * a.ldc + c;
          if (a.beta != 0.0) val += a.beta * (double)(*dst);
          *dst = (T)val;
        }
      }
}

template <typename T, int BM, int BN, int WM, int WN>
static hipError_t launch_regpf(const GemmArgs<T>& a, hipStream_t s) {
  if (a.K > 256) return hipErrorInvalidValue;
  const dim3 grid(xcd_grid(((a.N + BN - 1) / BN) * ((a.M + BM - 1) / BM), a.batch));
  if (a.K <= 160) {
    hipLaunchKernelGGL((gemm_regpf_kernel<T, BM, BN, WM, WN, 10>), grid, dim3(WM * WN * 64), 0, s, a);
  } else {
    // a single-wave tile would need 256 K values per thread: it only takes K <= 160
    if constexpr (WM * WN == 1) return hipErrorInvalidValue;
    else hipLaunchKernelGGL((gemm_regpf_kernel<T, BM, BN, WM, WN, 16>), grid, dim3(WM * WN * 64), 0, s, a);
  }
  return hipGetLastError();
}

template <typename T, int FM, int FN, int W>
static hipError_t launch_direct(const GemmArgs<T>& a, hipStream_t s) {
  if (a.K > 256) return hipErrorInvalidValue;   // the inner scales sit in LDS
  constexpr int BM = 16 * FM * W, BN = 16 * FN;
  const dim3 grid(xcd_grid(((a.N + BN - 1) / BN) * ((a.M + BM - 1) / BM), a.batch)), block(W * 64);
  if (a.tA)
    if (a.tB) hipLaunchKernelGGL((gemm_direct_kernel<T, FM, FN, W, true, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((gemm_direct_kernel<T, FM, FN, W, true, false>), grid, block, 0, s, a);
  else if (a.tB) hipLaunchKernelGGL((gemm_direct_kernel<T, FM, FN, W, false, true>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((gemm_direct_kernel<T, FM, FN, W, false, false>), grid, block, 0, s, a);
  return hipGetLastError();
}

template <typename T, int BM, int BN>
static size_t fullk_lds(int K) { return sizeof(T) * (size_t)((K + 3) & ~3) * (BM + BN + 4); }

template <typename T, int BM, int BN, int WM, int WN>
static hipError_t launch_fullk(const GemmArgs<T>& a, hipStream_t s) {
  const size_t lds = fullk_lds<T, BM, BN>(a.K);
  if (lds > 150 * 1024) return hipErrorInvalidValue;
  const dim3 grid(xcd_grid(((a.N + BN - 1) / BN) * ((a.M + BM - 1) / BM), a.batch));
  hipLaunchKernelGGL((gemm_fullk_kernel<T, BM, BN, WM, WN>), grid, dim3(WM * WN * 64), lds, s, a);
  return hipGetLastError();
}

template <typename T, int BM, int BN, int WM, int WN>
static hipError_t launch_tile(const GemmArgs<T>& a, hipStream_t s) {
  if (a.K > 256) return hipErrorInvalidValue;   // the inner scales sit in LDS
  const dim3 grid(xcd_grid(((a.N + BN - 1) / BN) * ((a.M + BM - 1) / BM), a.batch)), block(WM * WN * 64);
  if (a.tA)
    if (a.tB) hipLaunchKernelGGL((gemm_kernel<T, BM, BN, WM, WN, true, true>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((gemm_kernel<T, BM, BN, WM, WN, true, false>), grid, block, 0, s, a);
  else if (a.tB) hipLaunchKernelGGL((gemm_kernel<T, BM, BN, WM, WN, false, true>), grid, block, 0, s, a);
  else hipLaunchKernelGGL((gemm_kernel<T, BM, BN, WM, WN, false, false>), grid, block, 0, s, a);
  return hipGetLastError();
}

// one launch when a and b have the same transpositions and neither is
// transposed; otherwise one after the other
template <typename T, int BM, int BN, int WM, int WN>
static hipError_t launch_pair_tile(const GemmArgs<T>& a, const GemmArgs<T>& b, hipStream_t s) {
  if (a.tA || a.tB || b.tA || b.tB || a.K > 256 || b.K > 256) {
    hipError_t e = launch_tile<T, BM, BN, WM, WN>(a, s);
    if (e != hipSuccess) return e;
    return launch_tile<T, BM, BN, WM, WN>(b, s);
  }
  const dim3 grid(xcd_grid(((a.N + BN - 1) / BN) * ((a.M + BM - 1) / BM), a.batch + b.batch));
  hipLaunchKernelGGL((gemm_pair_kernel<T, BM, BN, WM, WN, false, false>), grid, dim3(WM * WN * 64), 0, s, a, b);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_any(const GemmArgs<T>& a, int tile, hipStream_t s);

// a and b in one launch where both have the same M and N and the tile is a
// staged one; otherwise one after the other
template <typename T>
static hipError_t launch_pair_any(const GemmArgs<T>& a, const GemmArgs<T>& b, int tile, hipStream_t s) {
  const bool same = a.M == b.M && a.N == b.N && a.M > 0 && a.N > 0 && a.batch > 0 && b.batch > 0 &&
                    !(a.ks.v && a.K > 256) && !(b.ks.v && b.K > 256);
  if (same) switch (tile) {
      case TILE_32x32: return launch_pair_tile<T, 32, 32, 2, 2>(a, b, s);
      case TILE_48x48: return launch_pair_tile<T, 48, 48, 3, 1>(a, b, s);
      case TILE_16x64: return launch_pair_tile<T, 16, 64, 1, 4>(a, b, s);
      case TILE_64x64: return launch_pair_tile<T, 64, 64, 2, 2>(a, b, s);
      default: break;
    }
  hipError_t e = launch_any(a, tile, s);
  if (e != hipSuccess) return e;
  return launch_any(b, tile, s);
}

template <typename T>
static hipError_t launch_any(const GemmArgs<T>& a, int tile, hipStream_t s) {
  if (a.M <= 0 || a.N <= 0 || a.batch <= 0) return hipSuccess;
  if (a.ks.v && a.K > 256) return hipErrorInvalidValue;   // the inner scale is staged in LDS
  switch (tile) {
    case TILE_32x32: return launch_tile<T, 32, 32, 2, 2>(a, s);
    case TILE_48x48: return launch_tile<T, 48, 48, 3, 1>(a, s);
    case TILE_16x64: return launch_tile<T, 16, 64, 1, 4>(a, s);
    case TILE_FK_32x32: return launch_fullk<T, 32, 32, 1, 1>(a, s);
    case TILE_FK_48x48: return launch_fullk<T, 48, 48, 3, 1>(a, s);
    case TILE_FK_64x64: return launch_fullk<T, 64, 64, 2, 2>(a, s);
    case TILE_FK_32x64: return launch_fullk<T, 32, 64, 1, 2>(a, s);
    case TILE_PF_48x48: return launch_regpf<T, 48, 48, 3, 1>(a, s);
    case TILE_PF_64x64: return launch_regpf<T, 64, 64, 2, 2>(a, s);
    case TILE_PF_32x32: return launch_regpf<T, 32, 32, 1, 1>(a, s);
    case TILE_DX_48x48: return launch_direct<T, 1, 3, 3>(a, s);
    case TILE_DX_32x32: return launch_direct<T, 1, 2, 2>(a, s);
    case TILE_DX_64x64: return launch_direct<T, 1, 4, 4>(a, s);
    default: return launch_tile<T, 64, 64, 2, 2>(a, s);
  }
}

hipError_t launch_gemm(const GemmArgs<double>& a, int tile, hipStream_t s) { return launch_any(a, tile, s); }
hipError_t launch_gemm(const GemmArgs<float>& a, int tile, hipStream_t s) { return launch_any(a, tile, s); }
hipError_t launch_gemm_pair(const GemmArgs<double>& a, const GemmArgs<double>& b, int tile, hipStream_t s) {
  return launch_pair_any(a, b, tile, s);
}

bool gemm_tile_fits(int tile, int K, int precision) {
  const bool f = precision != 0;
  switch (tile) {
    case TILE_FK_32x32: return (f ? fullk_lds<float, 32, 32>(K) : fullk_lds<double, 32, 32>(K)) <= 150 * 1024;
    case TILE_FK_48x48: return (f ? fullk_lds<float, 48, 48>(K) : fullk_lds<double, 48, 48>(K)) <= 150 * 1024;
    case TILE_FK_64x64: return (f ? fullk_lds<float, 64, 64>(K) : fullk_lds<double, 64, 64>(K)) <= 150 * 1024;
    case TILE_FK_32x64: return (f ? fullk_lds<float, 32, 64>(K) : fullk_lds<double, 32, 64>(K)) <= 150 * 1024;
    case TILE_PF_48x48:
    case TILE_PF_64x64: return K <= 256;
    case TILE_PF_32x32: return K <= 160;
    default: return K <= 256;               // the staged and direct tiles hold the inner scales in LDS
  }
}

template <typename T>
static hipError_t allow_fullk_t() {
  hipError_t e = hipSuccess, x;
  x = hipFuncSetAttribute((const void*)gemm_fullk_kernel<T, 32, 32, 1, 1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          150 * 1024);
  if (x != hipSuccess) e = x;
  x = hipFuncSetAttribute((const void*)gemm_fullk_kernel<T, 48, 48, 3, 1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          150 * 1024);
  if (x != hipSuccess) e = x;
  x = hipFuncSetAttribute((const void*)gemm_fullk_kernel<T, 64, 64, 2, 2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          150 * 1024);
  if (x != hipSuccess) e = x;
  x = hipFuncSetAttribute((const void*)gemm_fullk_kernel<T, 32, 64, 1, 2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          150 * 1024);
  if (x != hipSuccess) e = x;
  return e;
}

// ---------------------------------------------------------------------------
// Both products of a wrap in one launch:
//   G' = diag(rs2) (A1 diag(ks1) G diag(cs1)) A2 diag(cs2)
// with A1, A2 shared by the batch.  Two workgroups per chain split the rows
// of G' (tile rows [0, h0) and [h0, nt)); each forms its rows of the middle
// product X = A1 diag(ks1) G diag(cs1) in MFMA accumulators, parks them in
// LDS, and multiplies them by A2 streamed in 16-row chunks.  G is read once
// and G' written once, instead of a round trip of X through HBM.  Every
// workgroup reads all of G, so G' goes to a different buffer.
// ---------------------------------------------------------------------------
constexpr int WRAP_WAVES = 8;

// K advances in chunks of BK = 16
template <typename T> struct WrapBK { static constexpr int v = 16; };

template <typename T, int MAXT>
struct WrapLds {
  static constexpr int BK = WrapBK<T>::v;
  static constexpr int RTM = (MAXT + 1) / 2;     // tile rows of the larger half
  static constexpr int KP = (16 * MAXT + BK - 1) / BK * BK;   // columns of X, padded to whole chunks
  static constexpr int LDA = 16 * RTM + 1;       // A1 chunk, [k][local row]
  static constexpr int LDB = 16 * MAXT + 1;      // G / A2 chunks, [k][col]
  static constexpr int LDX = KP + 1;             // X, [row][col]
  static constexpr size_t bytes() { return sizeof(T) * ((size_t)2 * BK * LDA + 2 * BK * LDB + 16 * RTM * LDX); }
};

template <typename T, int MAXT>
__global__ __launch_bounds__(64 * WRAP_WAVES) void wrap_fused_kernel(WrapArgs<T> w) {
  typedef WrapLds<T, MAXT> Lay;
  constexpr int NT = 64 * WRAP_WAVES;
  constexpr int BK = Lay::BK, RTM = Lay::RTM, LDA = Lay::LDA, LDB = Lay::LDB, LDX = Lay::LDX;
  // output tiles per wave: wave w takes tile column w in every tile row (its
  // B values are shared by those tiles), and with nine tile columns wave w
  // also takes tile (w, 8)
  static_assert(MAXT <= WRAP_WAVES + 1, "one tile column per wave, plus one shared column");
  constexpr int TPW = RTM + (MAXT > WRAP_WAVES ? 1 : 0);
  constexpr int PA = (16 * RTM * BK + NT - 1) / NT;                  // A1 loads per thread per chunk
  constexpr int PB = (BK * 16 * MAXT + NT - 1) / NT;                 // G / A2 loads per thread per chunk
  extern __shared__ __align__(16) unsigned char smem[];
  T* As = (T*)smem;                        // [2][BK][LDA]
  T* Bs = As + 2 * BK * LDA;               // [2][BK][LDB]
  T* Xs = Bs + 2 * BK * LDB;               // [16 RTM][LDX]
  __shared__ double ksv[16 * MAXT], c1v[16 * MAXT], c2v[16 * MAXT], r2v[16 * RTM];

  const int n = w.n, nt = (n + 15) / 16;
  const int nch = (16 * nt + BK - 1) / BK;  // chunks per product
  int z, part;
  if (!xcd_tile(2, w.batch, z, part)) return;
  const int h0 = (nt + 1) / 2;
  const int t0 = part == 0 ? 0 : h0, nrt = part == 0 ? h0 : nt - h0;
  const int r0 = 16 * t0, R = 16 * nrt;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const T* G = w.Gin + (long)z * w.sG;
  T* Go = w.Gout + (long)z * w.sG;
  for (int i = tid; i < 16 * MAXT; i += NT) {
    ksv[i] = (i < n) ? scale_value(w.ks1, z, 1, i) : 0.0;
    c1v[i] = (i < n) ? scale_value(w.cs1, z, 1, i) : 0.0;
    c2v[i] = (i < n) ? scale_value(w.cs2, z, 1, i) : 0.0;
  }
  for (int i = tid; i < 16 * RTM; i += NT) r2v[i] = (i < R && r0 + i < n) ? scale_value(w.rs2, z, 1, r0 + i) : 0.0;
  // X columns past the last tile meet zero rows of A2 but must not hold stale values
  for (int e = tid; e < 16 * RTM * LDX; e += NT) Xs[e] = T(0);

  // the output tiles of this wave: tile rows trs (local), tile columns tcs
  int trs[TPW], tcs[TPW];
  bool own[TPW];
#pragma unroll
  for (int s = 0; s < TPW; ++s) {
    if (s < RTM) {
      trs[s] = s;
      tcs[s] = wave;
      own[s] = s < nrt && wave < nt;
    } else {
      trs[s] = wave;
      tcs[s] = WRAP_WAVES;
      own[s] = wave < nrt && WRAP_WAVES < nt;
    }
  }
  typedef typename Frag<T>::type F;
  F acc[TPW];
#pragma unroll
  for (int s = 0; s < TPW; ++s) acc[s] = F{0, 0, 0, 0};
  T ra[PA], rb[PB];
  // stage 1 chunk c: A1 rows r0 .. r0 + R, columns BK c ..; G rows BK c .., all columns
  auto load1 = [&](int c) {
#pragma unroll
    for (int q = 0; q < PA; ++q) {
      const int e = tid + NT * q, m = e / BK, k = e % BK, gk = BK * c + k;
      ra[q] = (m < R && r0 + m < n && gk < n) ? w.A1[(long)(r0 + m) * n + gk] : T(0);
    }
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      const int e = tid + NT * q, k = e / (16 * MAXT), col = e % (16 * MAXT), gk = BK * c + k;
      rb[q] = (k < BK && col < n && gk < n) ? G[(long)gk * n + col] : T(0);
    }
  };
  auto store1 = [&](int c, int buf) {
#pragma unroll
    for (int q = 0; q < PA; ++q) {
      const int e = tid + NT * q, m = e / BK, k = e % BK;
      if (m < 16 * RTM) As[(buf * BK + k) * LDA + m] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      const int e = tid + NT * q, k = e / (16 * MAXT), col = e % (16 * MAXT), gk = BK * c + k;
      if (k < BK) Bs[(buf * BK + k) * LDB + col] = (gk < n) ? (T)((double)rb[q] * ksv[gk] * c1v[col]) : T(0);
    }
  };
  // stage 2 chunk c: A2 rows BK c .., all columns
  auto load2 = [&](int c) {
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      const int e = tid + NT * q, k = e / (16 * MAXT), col = e % (16 * MAXT), gk = BK * c + k;
      rb[q] = (k < BK && col < n && gk < n) ? w.A2[(long)gk * n + col] : T(0);
    }
  };
  auto store2 = [&](int buf) {
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      const int e = tid + NT * q, k = e / (16 * MAXT), col = e % (16 * MAXT);
      if (k < BK) Bs[(buf * BK + k) * LDB + col] = rb[q];
    }
  };

  load1(0);
  __syncthreads();                         // scales
  store1(0, 0);
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    const int buf = c & 1;
    if (c + 1 < nch) load1(c + 1);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
#pragma unroll
      for (int s = 0; s < TPW; ++s)
        if (own[s]) {
          const T a = As[(buf * BK + kk + lk) * LDA + 16 * trs[s] + li];
          const T b = Bs[(buf * BK + kk + lk) * LDB + 16 * tcs[s] + li];
          acc[s] = mfma16(a, b, acc[s]);
        }
    }
    if (c + 1 < nch) store1(c + 1, buf ^ 1);   // buffer buf ^ 1 was last read before the previous barrier
    __syncthreads();
  }
  // X to LDS, row-major; the accumulators start over for G'
#pragma unroll
  for (int s = 0; s < TPW; ++s) {
    if (own[s]) {
#pragma unroll
      for (int v = 0; v < 4; ++v) Xs[(16 * trs[s] + frag_row<T>(lane, v)) * LDX + 16 * tcs[s] + li] = acc[s][v];
    }
    acc[s] = F{0, 0, 0, 0};
  }
  load2(0);
  store2(0);
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    const int buf = c & 1;
    if (c + 1 < nch) load2(c + 1);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
#pragma unroll
      for (int s = 0; s < TPW; ++s)
        if (own[s]) {
          const T a = Xs[(16 * trs[s] + li) * LDX + BK * c + kk + lk];
          const T b = Bs[(buf * BK + kk + lk) * LDB + 16 * tcs[s] + li];
          acc[s] = mfma16(a, b, acc[s]);
        }
    }
    if (c + 1 < nch) store2(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int s = 0; s < TPW; ++s)
    if (own[s]) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int lr = 16 * trs[s] + frag_row<T>(lane, v), col = 16 * tcs[s] + li;
        if (r0 + lr < n && col < n) Go[(long)(r0 + lr) * n + col] = (T)(r2v[lr] * (double)acc[s][v] * c2v[col]);
      }
    }
}

template <typename T, int MAXT>
static hipError_t launch_wrap_t(const WrapArgs<T>& w, hipStream_t s) {
  const size_t lds = WrapLds<T, MAXT>::bytes();
  hipLaunchKernelGGL((wrap_fused_kernel<T, MAXT>), dim3(xcd_grid(2, w.batch)), dim3(64 * WRAP_WAVES), lds, s, w);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_wrap_any(const WrapArgs<T>& w, hipStream_t s) {
  if (w.batch <= 0) return hipSuccess;
  if (!wrap_fused_supported(w.n, sizeof(T) == 4)) return hipErrorInvalidValue;
  if (w.n <= 64) return launch_wrap_t<T, 4>(w, s);
  if (w.n <= 112) return launch_wrap_t<T, 7>(w, s);
  return launch_wrap_t<T, 9>(w, s);
}

bool wrap_fused_supported(int n, bool fp32) {
  (void)fp32;
  return n >= 1 && n <= 144;
}
hipError_t launch_wrap_fused(const WrapArgs<double>& w, hipStream_t s) { return launch_wrap_any(w, s); }
hipError_t launch_wrap_fused(const WrapArgs<float>& w, hipStream_t s) { return launch_wrap_any(w, s); }

template <typename T>
static hipError_t allow_wrap_t() {
  hipError_t e = hipSuccess, x;
  x = hipFuncSetAttribute((const void*)wrap_fused_kernel<T, 4>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)WrapLds<T, 4>::bytes());
  if (x != hipSuccess) e = x;
  x = hipFuncSetAttribute((const void*)wrap_fused_kernel<T, 7>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)WrapLds<T, 7>::bytes());
  if (x != hipSuccess) e = x;
  x = hipFuncSetAttribute((const void*)wrap_fused_kernel<T, 9>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)WrapLds<T, 9>::bytes());
  if (x != hipSuccess) e = x;
  return e;
}

// raise the dynamic-LDS limit of the full-K kernels once, before any capture
hipError_t prepare_gemm() {
  const hipError_t e1 = allow_fullk_t<double>();
  const hipError_t e2 = allow_fullk_t<float>();
  const hipError_t e3 = allow_wrap_t<double>();
  const hipError_t e4 = allow_wrap_t<float>();
  return e1 != hipSuccess ? e1 : (e2 != hipSuccess ? e2 : (e3 != hipSuccess ? e3 : e4));
}

}  // namespace hq
