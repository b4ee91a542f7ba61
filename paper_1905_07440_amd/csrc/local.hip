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
// Thread j owns row j of A and Bv in registers and the running diagonal
// G_cur[j][j].  The random numbers and the bosonic action change of every
// site are independent of G, so each thread prepares its own site up front;
// the sequential part is one decision per site: the owner thread decides and
// publishes (accept, delta/r, its A and Bv rows) through a double-buffered
// LDS slot, one barrier, and on accept every thread extends its A/Bv row.
#include "hq_device.h"
#include "hq_internal.h"

namespace hq {

__host__ __device__ inline int lds_ld(int n) { return (n % 2 == 0) ? n + 1 : n; }
__host__ __device__ inline int pad16(int n) { return (n + 15) / 16 * 16; }

template <typename T>
__host__ __device__ inline size_t local_lds_size(int n, int kd) {
  return 128 + 16 + sizeof(T) * (size_t)(2 * (2 + 2 * kd) + n * lds_ld(n) + 2 * kd * pad16(n));
}

template <typename T, int NT, int KD>
__device__ inline void flush_lazy(T* G0, int ld, T* Ab, T* Bb, int n, int np, int m,
                                  T (&Ar)[KD], T (&Br)[KD]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NW = NT / 64;
  if (tid < np) {
#pragma unroll
    for (int k = 0; k < KD; ++k) {
      Ab[k * np + tid] = -Ar[k];
      Bb[k * np + tid] = Br[k];
    }
  }
  __syncthreads();
  typedef typename Frag<T>::type F;
  const int nt = np / 16;
  const int mm = (m + 3) & ~3;
  for (int t = wave; t < nt * nt; t += NW) {
    const int ti = t / nt, tj = t - ti * nt;
    const int cc = tj * 16 + (lane & 15);
    F acc;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = ti * 16 + frag_row<T>(lane, v);
      acc[v] = (r < n && cc < n) ? G0[r * ld + cc] : T(0);
    }
    for (int k0 = 0; k0 < mm; k0 += 4) {
      const T av = Ab[(k0 + (lane >> 4)) * np + ti * 16 + (lane & 15)];
      const T bv = Bb[(k0 + (lane >> 4)) * np + tj * 16 + (lane & 15)];
      acc = mfma16(av, bv, acc);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = ti * 16 + frag_row<T>(lane, v);
      if (r < n && cc < n) G0[r * ld + cc] = acc[v];
    }
  }
  __syncthreads();
}

template <typename T, int NT, int KD>
__global__ __launch_bounds__(NT) void local_slice_kernel(LocalArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = a.n, L = a.L, s = a.slice;
  const int np = pad16(n), ld = lds_ld(n);
  const int c = blockIdx.x;
  const int tid = threadIdx.x;

  double* red = (double*)smem;             // 16 doubles
  int* bflag = (int*)(red + 16);           // 4 ints
  T* bc = (T*)(bflag + 4);                 // 2 x [coef, pad, A[KD], B[KD]]
  T* G0 = bc + 2 * (2 + 2 * KD);
  T* Ab = G0 + n * ld;
  T* Bb = Ab + KD * np;

  const T* Gg = (const T*)a.G + (long)c * n * n;
  for (int e = tid; e < n * n; e += NT) {
    const int r = e / n, q = e - r * n;
    G0[r * ld + q] = Gg[e];
  }

  // ---- per-site preparation (independent of G) ----
  const int64_t sweep = *a.sweep;
  const int gchain = a.chain0 + c;
  double* x = a.x + (long)c * L * n;
  double d = 0.0, delta = 0.0, bos = 0.0, u1 = 2.0;
  uint8_t rp = 255;
  if (tid < n) {
    const Philox4 rn = philox4x64_10((uint64_t)gchain, (uint64_t)sweep, (uint64_t)(s * n + tid),
                                     KIND_LOCAL, a.seed, 0);
    const double u0 = u53(rn.w[0]);
    u1 = u53(rn.w[1]);
    d = a.width * (2.0 * u0 - 1.0);
    const double g = a.g[c];
    delta = expm1(-a.dtau * g * d);
    const double xa = x[s * n + tid];
    const double xprev = x[((s - 1 + L) % L) * n + tid];
    const double xnext = x[((s + 1) % L) * n + tid];
    const double kin = (a.mass / a.dtau) * (d * (2.0 * xa - xprev - xnext) + d * d);
    const double pot = a.dtau * 0.5 * a.mass * a.omega * a.omega * (2.0 * xa * d + d * d);
    bos = exp(-(kin + pot - a.dtau * g * d));
    if (a.replay) rp = a.replay[(long)c * L * n + s * n + tid];
  }
  __syncthreads();

  T diag = (tid < n) ? G0[tid * ld + tid] : T(0);
  T Ar[KD], Br[KD];
#pragma unroll
  for (int k = 0; k < KD; ++k) { Ar[k] = T(0); Br[k] = T(0); }
  int m = 0;
  double logr = 0.0;
  int nacc = 0, novr = 0, nmis = 0;

  for (int i = 0; i < n; ++i) {
    const int buf = i & 1;
    T* slot = bc + buf * (2 + 2 * KD);
    if (tid == i) {
      const double r = 1.0 + delta * (1.0 - (double)diag);
      const double R = r * r * bos;
      int acc = (u1 < R) ? 1 : 0;
      if (rp != 255 || a.log_margin) {
        const double margin = log(u1) - log(R);
        if (rp != 255) {
          if (fabs(margin) <= a.band) {
            if (acc != (int)rp) ++novr;
            acc = rp;
          } else if (acc != (int)rp) {
            ++nmis;
          }
        }
        if (a.log_margin) {
          const long o = (long)c * L * n + s * n + i;
          a.log_margin[o] = (float)margin;
          a.log_accept[o] = (uint8_t)acc;
        }
      }
      bflag[buf] = acc;
      slot[0] = (T)(delta / r);
#pragma unroll
      for (int k = 0; k < KD; ++k) { slot[2 + k] = Ar[k]; slot[2 + KD + k] = Br[k]; }
      if (acc) {
        x[s * n + i] += d;
        logr += log(fabs(r));
        ++nacc;
      }
    }
    __syncthreads();
    if (bflag[buf]) {
      const T coef = slot[0];
      T colv = T(0), rowv = T(0);
      if (tid < n) { colv = G0[tid * ld + i]; rowv = G0[i * ld + tid]; }
#pragma unroll
      for (int kc = 0; kc < KD; kc += 4) {
        if (kc < m) {
#pragma unroll
          for (int k = kc; k < kc + 4; ++k) {
            colv -= Ar[k] * slot[2 + KD + k];
            rowv -= slot[2 + k] * Br[k];
          }
        }
      }
      T na = coef * colv;
      T nb = ((tid == i) ? T(1) : T(0)) - rowv;
      if (tid >= n) { na = T(0); nb = T(0); }
#pragma unroll
      for (int k = 0; k < KD; ++k)
        if (k == m) { Ar[k] = na; Br[k] = nb; }
      diag -= na * nb;
      ++m;
      if (m == KD) {
        flush_lazy<T, NT, KD>(G0, ld, Ab, Bb, n, np, m, Ar, Br);
#pragma unroll
        for (int k = 0; k < KD; ++k) { Ar[k] = T(0); Br[k] = T(0); }
        m = 0;
        diag = (tid < n) ? G0[tid * ld + tid] : T(0);
      }
    }
  }
  if (m > 0) flush_lazy<T, NT, KD>(G0, ld, Ab, Bb, n, np, m, Ar, Br);

  T* Gw = (T*)a.G + (long)c * n * n;
  for (int e = tid; e < n * n; e += NT) {
    const int r = e / n, q = e - r * n;
    Gw[e] = G0[r * ld + q];
  }

  const double tot_logr = block_sum<NT>(logr, red);
  const double tot_acc = block_sum<NT>((double)nacc, red);
  const double tot_ovr = block_sum<NT>((double)novr, red);
  const double tot_mis = block_sum<NT>((double)nmis, red);
  if (tid == 0) {
    a.logdet[c] += tot_logr;
    int64_t* cnt = a.counters + (long)c * N_COUNTERS;
    cnt[CNT_LOCAL_P] += n;
    cnt[CNT_LOCAL_A] += (int64_t)tot_acc;
    if (a.replay_counts) {
      a.replay_counts[2 * c] += (int64_t)tot_ovr;
      a.replay_counts[2 * c + 1] += (int64_t)tot_mis;
    }
  }
}

size_t local_lds_bytes(int n, int precision, int nt, int kd) {
  (void)nt;
  return precision ? local_lds_size<float>(n, kd) : local_lds_size<double>(n, kd);
}

bool local_supported(int n, int precision, int nt, int kd) {
  if (n > nt || (nt != 64 && nt != 256) || (kd != 8 && kd != 16 && kd != 32)) return false;
  return local_lds_bytes(n, precision, nt, kd) <= 160 * 1024;
}

template <typename T, int NT, int KD>
static hipError_t launch_local_t(const LocalArgs& a, int chains, hipStream_t s) {
  const size_t lds = local_lds_size<T>(a.n, KD);
  hipLaunchKernelGGL((local_slice_kernel<T, NT, KD>), dim3(chains), dim3(NT), lds, s, a);
  return hipGetLastError();
}

template <typename T, int NT, int KD>
static hipError_t allow_lds() {
  return hipFuncSetAttribute((const void*)local_slice_kernel<T, NT, KD>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

// raise the dynamic-LDS limit of every instantiation once, before any capture
hipError_t prepare_local() {
  hipError_t e = hipSuccess;
  const hipError_t all[] = {
      allow_lds<double, 64, 8>(), allow_lds<double, 64, 16>(), allow_lds<double, 64, 32>(),
      allow_lds<double, 256, 8>(), allow_lds<double, 256, 16>(), allow_lds<double, 256, 32>(),
      allow_lds<float, 64, 8>(), allow_lds<float, 64, 16>(), allow_lds<float, 64, 32>(),
      allow_lds<float, 256, 8>(), allow_lds<float, 256, 16>(), allow_lds<float, 256, 32>()};
  for (hipError_t x : all)
    if (x != hipSuccess) e = x;
  return e;
}

template <typename T>
static hipError_t launch_local_p(const LocalArgs& a, int nt, int kd, int chains, hipStream_t s) {
  if (nt == 64) {
    if (kd == 8) return launch_local_t<T, 64, 8>(a, chains, s);
    if (kd == 16) return launch_local_t<T, 64, 16>(a, chains, s);
    return launch_local_t<T, 64, 32>(a, chains, s);
  }
  if (kd == 8) return launch_local_t<T, 256, 8>(a, chains, s);
  if (kd == 16) return launch_local_t<T, 256, 16>(a, chains, s);
  return launch_local_t<T, 256, 32>(a, chains, s);
}

hipError_t launch_local(const LocalArgs& a, int precision, int nt, int kd, int chains, hipStream_t s) {
  if (!local_supported(a.n, precision, nt, kd)) return hipErrorInvalidValue;
  return precision ? launch_local_p<float>(a, nt, kd, chains, s)
                   : launch_local_p<double>(a, nt, kd, chains, s);
}

}  // namespace hq
