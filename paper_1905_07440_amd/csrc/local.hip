// Local moves of one imaginary-time slice: the sequential Metropolis chain
// over the N sites of slice l, with delayed rank-k updates of G.
//
// Paper, section "Determinant quantum Monte Carlo": a local move changes
// one X_{i,l}; it is accepted with W'/W.  With B_l' = (I + Delta) B_l,
// Delta = delta e_i e_i^T, delta = exp(-dtau g d) - 1, and G the equal-time
// Green's function at slice l,
//     det ratio (one spin)  r = 1 + delta (1 - G_ii)
//     new G                 G' = G - (delta / r) G[:,i] (e_i - G[i,:])
// and W'/W = r^2 exp(-dS_b).
//
// Delayed form: G_cur = G0 - A Bv^T with A, Bv of width k.  An accepted move
// at site i appends A[:,m] = (delta/r) G_cur[:,i] and Bv[:,m] = e_i - G_cur[i,:]
// (both from G0 and the first m columns); after k accepts, or at the end of
// the slice, G0 <- G0 - A Bv^T as one rank-k MFMA product.
//
// Design: one workgroup per chain, G0 resident in LDS for the whole slice.
// The sites are visited by a single "walker" wave, so the sequential chain
// has no barriers at all: lane q owns rows q, q+64, q+128, ... -- their
// random numbers and bosonic action changes (prepared up front, since they do
// not depend on G), their running diagonal G_cur[j][j], and their rows of A
// and Bv in registers.  The decision for site i reads the owner lane's values
// with readlane and is taken by the whole wave; on accept, row i of A and Bv
// is broadcast the same way and every lane extends its rows.  The other three
// waves sleep at a barrier and join only for the rank-k flushes, which read A
// and Bv from LDS mirrors the walker keeps up to date.
#include "hq_device.h"
#include "hq_internal.h"

namespace hq {

__host__ __device__ inline int lds_ld(int n) { return (n % 2 == 0) ? n + 1 : n; }
__host__ __device__ inline int pad16(int n) { return (n + 15) / 16 * 16; }
// G0 occupies n * ld elements, rounded up so that the mirrors after it are 16-byte aligned
__host__ __device__ inline int g0_elems(int n) { return (n * lds_ld(n) + 3) / 4 * 4; }
template <typename T, int KD> struct Mirror { enum { ld = KD + 16 / (int)sizeof(T) }; };

__host__ __device__ inline int site_table_len(int n) { return n <= 64 ? 64 : (n <= 192 ? 192 : 256); }

template <typename T, int KD>
__host__ __device__ inline size_t local_lds_size(int n) {
  return 64 + 32 * (size_t)site_table_len(n) + sizeof(T) * (size_t)(g0_elems(n) + 2 * pad16(n) * Mirror<T, KD>::ld);
}

__device__ inline int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline float bcast(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ inline double bcast(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// G0 <- G0 - A Bv^T over the first m columns (all four waves; tiles split by wave)
template <typename T, int KD>
__device__ inline void flush_tiles(T* G0, int ld, const T* Am, const T* Bm, int n, int np, int m) {
  constexpr int KL = Mirror<T, KD>::ld;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  typedef typename Frag<T>::type F;
  const int nt = np / 16;
  const int mm = (m + 3) & ~3;
  for (int t = wave; t < nt * nt; t += 4) {
    const int ti = t / nt, tj = t - ti * nt;
    const int cc = tj * 16 + (lane & 15);
    F acc;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = ti * 16 + frag_row<T>(lane, v);
      acc[v] = (r < n && cc < n) ? G0[r * ld + cc] : T(0);
    }
    for (int k0 = 0; k0 < mm; k0 += 4) {
      const T av = -Am[(ti * 16 + (lane & 15)) * KL + k0 + (lane >> 4)];
      const T bv = Bm[(tj * 16 + (lane & 15)) * KL + k0 + (lane >> 4)];
      acc = mfma16(av, bv, acc);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = ti * 16 + frag_row<T>(lane, v);
      if (r < n && cc < n) G0[r * ld + cc] = acc[v];
    }
  }
}

// per-site constants of the slice, prepared by the owner lane: delta,
// exp(-dS_b), u, replay bit (255 = none)
struct SiteConst { double delta, bos, u, rp; };

template <typename T, int RPL>
__device__ inline T pick(const T (&v)[RPL], int t) {
  T r = v[0];
#pragma unroll
  for (int q = 1; q < RPL; ++q) r = (t == q) ? v[q] : r;
  return r;
}

template <typename T> struct Vec;
template <> struct Vec<float> { typedef float4 type; enum { w = 4 }; };
template <> struct Vec<double> { typedef double2 type; enum { w = 2 }; };

// sum_{q<m} a[q] * b[q] for a, b in LDS (16-byte aligned rows)
template <typename T>
__device__ __forceinline__ T dot_lds(const T* a, const T* b, int m) {
  typedef typename Vec<T>::type V;
  constexpr int W = Vec<T>::w;
  T s0 = T(0), s1 = T(0);
  for (int q = 0; q < m; q += W) {
    const V va = *(const V*)(a + q);
    const V vb = *(const V*)(b + q);
    if constexpr (W == 4) {
      s0 += va.x * vb.x;
      s1 += va.y * vb.y;
      s0 += va.z * vb.z;
      s1 += va.w * vb.w;
    } else {
      s0 += va.x * vb.x;
      s1 += va.y * vb.y;
    }
  }
  return s0 + s1;
}

template <typename T, int KD, int RPL>
__global__ __launch_bounds__(256) void local_slice_kernel(LocalArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int KL = Mirror<T, KD>::ld;
  constexpr int MAXN = 64 * RPL;
  const int n = a.n, L = a.L, s = a.slice;
  const int np = pad16(n), ld = lds_ld(n);
  const int c = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  int* cmd = (int*)smem;                   // flush command: m > 0 flush, -1 done
  SiteConst* sc = (SiteConst*)(smem + 64);
  T* G0 = (T*)(smem + 64 + sizeof(SiteConst) * MAXN);
  T* Am = G0 + g0_elems(n);                // [np][KL] row-major A and Bv (entries >= m are zero)
  T* Bm = Am + np * KL;

  const T* Gg = (const T*)a.G + (long)c * n * n;
  batched_copy<256, 16, T>(n * n, [&](int e) { return Gg[e]; },
                           [&](int e, T v) { const int r = e / n; G0[r * ld + (e - r * n)] = v; });
  for (int e = tid; e < 2 * np * KL; e += 256) Am[e] = T(0);

  double* x = a.x + (long)c * L * n;
  double d[RPL], xold[RPL];
  if (wave == 0) {
    const int64_t sweep = *a.sweep;
    const double g = a.g[c];
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int j = lane + 64 * t;
      d[t] = 0.0;
      xold[t] = 0.0;
      if (j < n) {
        const double xa = x[s * n + j];
        const double xprev = x[((s - 1 + L) % L) * n + j];
        const double xnext = x[((s + 1) % L) * n + j];
        const Philox4 rn = philox4x64_10((uint64_t)(a.chain0 + c), (uint64_t)sweep, (uint64_t)(s * n + j),
                                         KIND_LOCAL, a.seed, 0);
        d[t] = a.width * (2.0 * u53(rn.w[0]) - 1.0);
        const double kin = (a.mass / a.dtau) * (d[t] * (2.0 * xa - xprev - xnext) + d[t] * d[t]);
        const double pot = a.dtau * 0.5 * a.mass * a.omega * a.omega * (2.0 * xa * d[t] + d[t] * d[t]);
        SiteConst k;
        k.delta = expm1(-a.dtau * g * d[t]);
        k.bos = exp(-(kin + pot - a.dtau * g * d[t]));
        k.u = u53(rn.w[1]);
        k.rp = a.replay ? (double)a.replay[(long)c * L * n + s * n + j] : 255.0;
        sc[j] = k;
        xold[t] = xa;
      }
    }
  }
  __syncthreads();

  double logr = 0.0;
  int nacc = 0, novr = 0, nmis = 0;
  if (wave != 0) {
    // helpers: wake for each flush the walker requests
    while (true) {
      __syncthreads();
      const int m = cmd[0];
      if (m < 0) break;
      flush_tiles<T, KD>(G0, ld, Am, Bm, n, np, m);
      __syncthreads();
    }
  } else {
    // ---- walker ----
    T diag[RPL];
    float my_margin[RPL];
    int my_acc = 0;                        // bit t: site lane + 64 t accepted
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int j = lane + 64 * t;
      diag[t] = (j < n) ? G0[j * ld + j] : T(0);
      my_margin[t] = 0.0f;
    }
    const bool logging = (a.log_margin != nullptr);
    int m = 0;
    SiteConst nxt = sc[0];
    for (int i = 0; i < n; ++i) {
      const SiteConst cur = nxt;
      if (i + 1 < n) nxt = sc[i + 1];
      const int t = i >> 6, o = i & 63;
      // decision for site i, taken by the whole wave from the owner lane's diagonal
      const double dg = (double)bcast(pick<T, RPL>(diag, t), o);
      const double r = 1.0 + cur.delta * (1.0 - dg);
      const double R = r * r * cur.bos;
      int acc = (cur.u < R) ? 1 : 0;
      const int rpi = (int)cur.rp;
      if (rpi != 255 || logging) {
        const double margin = log(cur.u) - log(R);
        if (rpi != 255) {
          if (fabs(margin) <= a.band) {
            if (acc != rpi) ++novr;
            acc = rpi;
          } else if (acc != rpi) {
            ++nmis;
          }
        }
        if (logging) {
#pragma unroll
          for (int q = 0; q < RPL; ++q)
            if (lane == o && t == q) my_margin[q] = (float)margin;
        }
      }
      if (!acc) continue;
      // accepted: site i becomes column m of A and Bv
      if (lane == o) my_acc |= 1 << t;
      logr += log(fabs(r));
      ++nacc;
      const T coef = (T)(cur.delta / r);
      const T* ai = Am + i * KL;           // row i (broadcast: every lane reads the same address)
      const T* bi = Bm + i * KL;
#pragma unroll
      for (int t2 = 0; t2 < RPL; ++t2) {
        const int j = lane + 64 * t2;
        if (j < np) {
          const T colv = ((j < n) ? G0[j * ld + i] : T(0)) - dot_lds<T>(Am + j * KL, bi, m);
          const T rowv = ((j < n) ? G0[i * ld + j] : T(0)) - dot_lds<T>(ai, Bm + j * KL, m);
          T na = coef * colv;
          T nb = ((j == i) ? T(1) : T(0)) - rowv;
          if (j >= n) { na = T(0); nb = T(0); }
          diag[t2] -= na * nb;
          // the dots of every lane read row i before any lane writes column m
          __builtin_amdgcn_wave_barrier();
          Am[j * KL + m] = na;
          Bm[j * KL + m] = nb;
        }
      }
      m = uniform(m + 1);
      if (m == KD) {
        // window full: G0 <- G0 - A Bv^T with every wave, then a fresh window
        cmd[0] = KD;
        __syncthreads();
        flush_tiles<T, KD>(G0, ld, Am, Bm, n, np, KD);
        __syncthreads();
#pragma unroll
        for (int t2 = 0; t2 < RPL; ++t2) {
          const int j = lane + 64 * t2;
          if (j < np)
            for (int q = 0; q < KD; ++q) { Am[j * KL + q] = T(0); Bm[j * KL + q] = T(0); }
          diag[t2] = (j < n) ? G0[j * ld + j] : T(0);
        }
        m = 0;
      }
    }
    if (m > 0) {
      cmd[0] = m;
      __syncthreads();
      flush_tiles<T, KD>(G0, ld, Am, Bm, n, np, m);
      __syncthreads();
    }
    cmd[0] = -1;
    __syncthreads();
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int j = lane + 64 * t;
      if (j < n) {
        const bool acc = (my_acc >> t) & 1;
        if (acc) x[s * n + j] = xold[t] + d[t];
        if (logging) {
          const long o = (long)c * L * n + s * n + j;
          a.log_margin[o] = my_margin[t];
          a.log_accept[o] = (uint8_t)acc;
        }
      }
    }
  }
  __syncthreads();

  T* Gw = (T*)a.G + (long)c * n * n;
  batched_copy<256, 16, T>(n * n, [&](int e) { const int r = e / n; return G0[r * ld + (e - r * n)]; },
                           [&](int e, T v) { Gw[e] = v; });
  if (tid == 0) {
    a.logdet[c] += logr;
    int64_t* cnt = a.counters + (long)c * N_COUNTERS;
    cnt[CNT_LOCAL_P] += n;
    cnt[CNT_LOCAL_A] += nacc;
    if (a.replay_counts) {
      a.replay_counts[2 * c] += novr;
      a.replay_counts[2 * c + 1] += nmis;
    }
  }
}

template <int KD>
static size_t lds_for(int n, int precision) {
  return precision ? local_lds_size<float, KD>(n) : local_lds_size<double, KD>(n);
}

size_t local_lds_bytes(int n, int precision, int nt, int kd) {
  (void)nt;
  if (kd == 8) return lds_for<8>(n, precision);
  if (kd == 16) return lds_for<16>(n, precision);
  return lds_for<32>(n, precision);
}

bool local_supported(int n, int precision, int nt, int kd) {
  (void)nt;
  if (n < 1 || n > 256 || (kd != 8 && kd != 16 && kd != 32)) return false;
  if (!precision && kd == 32 && n > 64) return false;   // FP64, 3-4 rows per lane: at most 16 columns in registers
  return local_lds_bytes(n, precision, 256, kd) <= 160 * 1024;
}

template <typename T, int KD, int RPL>
static hipError_t launch_local_t(const LocalArgs& a, int chains, hipStream_t s) {
  const size_t lds = local_lds_size<T, KD>(a.n);
  hipLaunchKernelGGL((local_slice_kernel<T, KD, RPL>), dim3(chains), dim3(256), lds, s, a);
  return hipGetLastError();
}

template <typename T, int KD>
static hipError_t launch_local_k(const LocalArgs& a, int chains, hipStream_t s) {
  if (a.n <= 64) return launch_local_t<T, KD, 1>(a, chains, s);
  if constexpr (sizeof(T) == 8 && KD == 32) {
    return hipErrorInvalidValue;
  } else {
    if (a.n <= 192) return launch_local_t<T, KD, 3>(a, chains, s);
    return launch_local_t<T, KD, 4>(a, chains, s);
  }
}

template <typename T, int KD>
static hipError_t allow_lds_k() {
  hipError_t e = hipSuccess, x;
  x = hipFuncSetAttribute((const void*)local_slice_kernel<T, KD, 1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          160 * 1024);
  if (x != hipSuccess) e = x;
  if constexpr (!(sizeof(T) == 8 && KD == 32)) {
    x = hipFuncSetAttribute((const void*)local_slice_kernel<T, KD, 3>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
    if (x != hipSuccess) e = x;
    x = hipFuncSetAttribute((const void*)local_slice_kernel<T, KD, 4>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
    if (x != hipSuccess) e = x;
  }
  return e;
}

// raise the dynamic-LDS limit of every instantiation once, before any capture
hipError_t prepare_local() {
  hipError_t e = hipSuccess;
  const hipError_t all[] = {allow_lds_k<double, 8>(), allow_lds_k<double, 16>(), allow_lds_k<double, 32>(),
                            allow_lds_k<float, 8>(), allow_lds_k<float, 16>(), allow_lds_k<float, 32>()};
  for (hipError_t x : all)
    if (x != hipSuccess) e = x;
  return e;
}

hipError_t launch_local(const LocalArgs& a, int precision, int nt, int kd, int chains, hipStream_t s) {
  if (!local_supported(a.n, precision, nt, kd)) return hipErrorInvalidValue;
  if (precision) {
    if (kd == 8) return launch_local_k<float, 8>(a, chains, s);
    if (kd == 16) return launch_local_k<float, 16>(a, chains, s);
    return launch_local_k<float, 32>(a, chains, s);
  }
  if (kd == 8) return launch_local_k<double, 8>(a, chains, s);
  if (kd == 16) return launch_local_k<double, 16>(a, chains, s);
  return launch_local_k<double, 32>(a, chains, s);
}

}  // namespace hq
