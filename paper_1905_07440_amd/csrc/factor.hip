// FP64 dense factorizations for the stabilised recomputation of G.
//
// The paper defines G through M = I + B_L ... B_1 and refers to the standard
// DQMC literature for computing it without overflow: the running product is
// kept as U D T with a pivoted QR after every block of n_stab slices.  Two
// kernels serve that scheme, one workgroup per matrix, the matrix held in
// registers (thread = (column, row part); rows r = part + TPC*k):
//
//  qr_kernel  Householder QR of Z with columns pre-sorted by decreasing norm
//             (pre-pivoting: the column order is fixed before the
//             factorization, which keeps the graded scales of Z = (C U) D in
//             order without per-step pivot searches).  Outputs Q, D = |diag R|
//             and Rt = D^-1 R P^T, so Z = Q D Rt.
//  gj_kernel  in-place Gauss-Jordan inversion with partial (row) pivoting,
//             M^-1 scaled as diag(rs) M^-1 diag(cs), and log|det M|.
#include "hq_device.h"
#include "hq_internal.h"

namespace hq {

// value of the (column-group-shared) element at row `row`
template <int TPC, int RPT>
__device__ inline double pick_row(const double (&a)[RPT], int q, int row) {
  double v = 0.0;
#pragma unroll
  for (int k = 0; k < RPT; ++k) v = (q + TPC * k == row) ? a[k] : v;
  return group_sum<TPC>(v);
}

// ---------------------------------------------------------------------------
// QR with pre-pivoting
// ---------------------------------------------------------------------------
template <int TPC, int RPT, int MAXT>
__global__ __launch_bounds__(MAXT) void qr_kernel(const double* __restrict__ Zg, double* __restrict__ Qg,
                                                  double* __restrict__ Dg, double* __restrict__ Rtg, int n) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* norms = (double*)smem;          // n
  double* tau = norms + n;                // n
  double* beta = tau + n;                 // n
  int* perm = (int*)(beta + n);           // n
  double* vst = (double*)(perm + ((n + 1) & ~1));   // packed: v_j[r], r >= j, at off(j) + r - j
  const int z = blockIdx.x;
  const int tid = threadIdx.x;
  const int c = tid / TPC, q = tid % TPC;
  const bool live = c < n;
  const double* Z = Zg + (long)z * n * n;

  double a[RPT];
  // column norms of Z for the pre-pivoting order
  double ss = 0.0;
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int r = q + TPC * k;
    a[k] = (live && r < n) ? Z[(long)r * n + c] : 0.0;
    ss += a[k] * a[k];
  }
  ss = group_sum<TPC>(ss);
  if (!(ss == ss)) ss = -1.0;   // a NaN column sorts last; ranks stay a permutation
  if (live && q == 0) norms[c] = ss;
  __syncthreads();
  if (live && q == 0) {
    int rank = 0;
    for (int k = 0; k < n; ++k) {
      const double o = norms[k];
      rank += (o > ss || (o == ss && k < c)) ? 1 : 0;
    }
    perm[rank] = c;
  }
  __syncthreads();
  const int pc = live ? min(max(perm[c], 0), n - 1) : 0;
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int r = q + TPC * k;
    a[k] = (live && r < n) ? Z[(long)r * n + pc] : 0.0;
  }

  for (int j = 0; j < n; ++j) {
    const long off = (long)j * n - (long)j * (j - 1) / 2;   // start of v_j in the packed store
    if (live && c == j) {
      double sig = 0.0, alpha = 0.0;
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int r = q + TPC * k;
        if (r > j && r < n) sig += a[k] * a[k];
        if (r == j) alpha = a[k];
      }
      sig = group_sum<TPC>(sig);
      alpha = group_sum<TPC>(alpha);
      double t = 0.0, b = alpha, scl = 0.0;
      if (sig > 0.0) {
        const double nrm = sqrt(alpha * alpha + sig);
        b = (alpha >= 0.0) ? -nrm : nrm;
        t = (b - alpha) / b;
        scl = 1.0 / (alpha - b);
      }
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int r = q + TPC * k;
        if (r == j) { vst[off] = 1.0; a[k] = b; }
        else if (r > j && r < n) { vst[off + r - j] = a[k] * scl; }
      }
      if (q == 0) { tau[j] = t; beta[j] = b; }
    }
    __syncthreads();
    if (live && c > j) {
      const double t = tau[j];
      double w = 0.0;
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int r = q + TPC * k;
        if (r >= j && r < n) w += vst[off + r - j] * a[k];
      }
      w = group_sum<TPC>(w) * t;
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int r = q + TPC * k;
        if (r >= j && r < n) a[k] -= vst[off + r - j] * w;
      }
    }
  }
  __syncthreads();

  // D = |diag R|, Rt = D^-1 R P^T (column c of R goes to column perm[c])
  double* Rt = Rtg + (long)z * n * n;
  if (live) {
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int r = q + TPC * k;
      if (r < n) Rt[(long)r * n + pc] = (r <= c) ? a[k] / fabs(beta[r]) : 0.0;
    }
    if (q == 0) Dg[(long)z * n + c] = fabs(beta[c]);
  }

  // Q = H_0 H_1 ... H_{n-1}, accumulated backwards from the identity
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int r = q + TPC * k;
    a[k] = (live && r == c) ? 1.0 : 0.0;
  }
  for (int j = n - 1; j >= 0; --j) {
    if (live && c >= j) {
      const long off = (long)j * n - (long)j * (j - 1) / 2;
      const double t = tau[j];
      double w = 0.0;
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int r = q + TPC * k;
        if (r >= j && r < n) w += vst[off + r - j] * a[k];
      }
      w = group_sum<TPC>(w) * t;
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int r = q + TPC * k;
        if (r >= j && r < n) a[k] -= vst[off + r - j] * w;
      }
    }
  }
  double* Q = Qg + (long)z * n * n;
  if (live) {
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int r = q + TPC * k;
      if (r < n) Q[(long)r * n + c] = a[k];
    }
  }
}

static size_t qr_lds(int n) {
  return sizeof(double) * (3 * (size_t)n) + sizeof(int) * ((n + 1) & ~1) +
         sizeof(double) * ((size_t)n * (n + 1) / 2);
}

struct FactorCfg { int tpc, rpt, threads; };

static FactorCfg factor_cfg(int n) {
  FactorCfg f{0, 0, 0};
  if (n <= 16) f = {16, 1, 0};
  else if (n <= 32) f = {16, 2, 0};
  else if (n <= 64) f = {16, 4, 0};
  else if (n <= 128) f = {8, 16, 0};
  else if (n <= 144) f = {4, 36, 0};
  else if (n <= 192) f = {4, 48, 0};
  else return f;
  f.threads = (f.tpc * n + 63) / 64 * 64;
  return f;
}

bool qr_supported(int n) { return n >= 1 && factor_cfg(n).tpc > 0 && qr_lds(n) <= 160 * 1024; }

// largest block each register layout is launched with: TPC * max n, rounded to waves
template <int TPC, int RPT> struct MaxThreads { enum { value = (TPC * TPC * RPT + 63) / 64 * 64 }; };

template <int TPC, int RPT>
static hipError_t qr_launch_t(const double* Z, double* Q, double* D, double* Rt, int n, int batch,
                              int threads, hipStream_t s) {
  hipLaunchKernelGGL((qr_kernel<TPC, RPT, MaxThreads<TPC, RPT>::value>), dim3(batch), dim3(threads), qr_lds(n), s,
                     Z, Q, D, Rt, n);
  return hipGetLastError();
}

template <int TPC, int RPT>
static hipError_t qr_allow_lds() {
  return hipFuncSetAttribute((const void*)qr_kernel<TPC, RPT, MaxThreads<TPC, RPT>::value>,
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             160 * 1024);
}

hipError_t prepare_factor() {
  hipError_t e = hipSuccess;
  const hipError_t all[] = {qr_allow_lds<16, 1>(), qr_allow_lds<16, 2>(), qr_allow_lds<16, 4>(),
                            qr_allow_lds<8, 16>(), qr_allow_lds<4, 36>(), qr_allow_lds<4, 48>()};
  for (hipError_t x : all)
    if (x != hipSuccess) e = x;
  return e;
}

hipError_t launch_qr(const double* Z, double* Q, double* D, double* Rt, int n, int batch, hipStream_t s) {
  if (!qr_supported(n)) return hipErrorInvalidValue;
  const FactorCfg f = factor_cfg(n);
  switch (f.rpt) {
    case 1: return qr_launch_t<16, 1>(Z, Q, D, Rt, n, batch, f.threads, s);
    case 2: return qr_launch_t<16, 2>(Z, Q, D, Rt, n, batch, f.threads, s);
    case 4: return qr_launch_t<16, 4>(Z, Q, D, Rt, n, batch, f.threads, s);
    case 16: return qr_launch_t<8, 16>(Z, Q, D, Rt, n, batch, f.threads, s);
    case 36: return qr_launch_t<4, 36>(Z, Q, D, Rt, n, batch, f.threads, s);
    default: return qr_launch_t<4, 48>(Z, Q, D, Rt, n, batch, f.threads, s);
  }
}

// ---------------------------------------------------------------------------
// Gauss-Jordan inversion in place, partial pivoting
//
// Step j picks the unused row p with the largest |W[p][j]|, scales row p by
// 1/piv and eliminates column j from every other row; column j's storage then
// holds the column p of the accumulated inverse.  At the end
// M^-1[j][perm[k]] = W[perm[j]][k], perm[j] being the pivot row of step j.
// ---------------------------------------------------------------------------
template <int TPC, int RPT, int MAXT>
__global__ __launch_bounds__(MAXT) void gj_kernel(const double* __restrict__ Mg, double* __restrict__ Xg,
                                                  const double* __restrict__ rsg, const double* __restrict__ csg,
                                                  const double* __restrict__ base, double* __restrict__ logdet,
                                                  int n) {
  extern __shared__ __align__(16) unsigned char smem[];
  double* fbuf = (double*)smem;           // 2 x n: column j of W before step j
  double* red = fbuf + 2 * n;             // 2 x 2: pivot value, pivot index
  double* logp = red + 4;                 // n
  int* perm = (int*)(logp + n);           // n
  int* pinv = perm + n;                   // n
  int* used = pinv + n;                   // n
  const int z = blockIdx.x;
  const int tid = threadIdx.x;
  const int c = tid / TPC, q = tid % TPC;
  const bool live = c < n;
  const double* M = Mg + (long)z * n * n;

  double a[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int r = q + TPC * k;
    a[k] = (live && r < n) ? M[(long)r * n + c] : 0.0;
  }
  for (int e = tid; e < n; e += blockDim.x) used[e] = 0;
  __syncthreads();

  for (int j = 0; j < n; ++j) {
    double* f = fbuf + (j & 1) * n;
    double* rd = red + (j & 1) * 2;
    if (live && c == j) {
      double best = -1.0;
      int bi = n, fu = n;            // fu: first unused row, the fallback for a NaN column
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int r = q + TPC * k;
        if (r < n) {
          f[r] = a[k];
          const double v = fabs(a[k]);
          if (!used[r]) {
            fu = min(fu, r);
            if (v > best || (v == best && r < bi)) { best = v; bi = r; }
          }
        }
      }
#pragma unroll
      for (int o = TPC / 2; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        fu = min(fu, __shfl_xor(fu, o, 64));
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (bi >= n) bi = (fu < n) ? fu : 0;
      if (q == 0) { rd[1] = (double)bi; perm[j] = bi; pinv[bi] = j; used[bi] = 1; }
    }
    __syncthreads();
    const int p = (int)rd[1];
    const double piv = f[p];
    const double pinv_v = 1.0 / piv;
    if (live) {
      if (c == j) {
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
          const int r = q + TPC * k;
          a[k] = (r == p) ? pinv_v : -a[k] * pinv_v;
        }
      } else {
        const double wp = pick_row<TPC, RPT>(a, q, p) * pinv_v;
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
          const int r = q + TPC * k;
          a[k] = (r == p) ? wp : a[k] - f[r < n ? r : 0] * wp;
        }
      }
    }
    if (tid == 0) logp[j] = log(fabs(piv));
  }
  __syncthreads();

  // scatter: X[j][perm[k]] = rs[j] * W[perm[j]][k] * cs[perm[k]]
  if (live) {
    const int pk = perm[c];
    const double* rs = rsg + (long)z * n;
    const double* cs = csg + (long)z * n;
    double* X = Xg + (long)z * n * n;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int r = q + TPC * k;
      if (r < n) {
        const int jr = pinv[r];
        X[(long)jr * n + pk] = rs[jr] * a[k] * cs[pk];
      }
    }
  }
  if (tid == 0) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += logp[j];
    logdet[z] = base[z] + s;
  }
}

static size_t gj_lds(int n) { return sizeof(double) * (3 * (size_t)n + 4) + sizeof(int) * 4 * (size_t)n; }

bool gj_supported(int n) { return n >= 1 && factor_cfg(n).tpc > 0; }

template <int TPC, int RPT>
static hipError_t gj_launch_t(const double* M, double* X, const double* rs, const double* cs,
                              const double* base, double* logdet, int n, int batch, int threads,
                              hipStream_t s) {
  hipLaunchKernelGGL((gj_kernel<TPC, RPT, MaxThreads<TPC, RPT>::value>), dim3(batch), dim3(threads), gj_lds(n), s,
                     M, X, rs, cs, base, logdet, n);
  return hipGetLastError();
}

hipError_t launch_gj(const double* M, double* X, const double* rs, const double* cs, const double* base,
                     double* logdet, int n, int batch, hipStream_t s) {
  if (!gj_supported(n)) return hipErrorInvalidValue;
  const FactorCfg f = factor_cfg(n);
  switch (f.rpt) {
    case 1: return gj_launch_t<16, 1>(M, X, rs, cs, base, logdet, n, batch, f.threads, s);
    case 2: return gj_launch_t<16, 2>(M, X, rs, cs, base, logdet, n, batch, f.threads, s);
    case 4: return gj_launch_t<16, 4>(M, X, rs, cs, base, logdet, n, batch, f.threads, s);
    case 16: return gj_launch_t<8, 16>(M, X, rs, cs, base, logdet, n, batch, f.threads, s);
    case 36: return gj_launch_t<4, 36>(M, X, rs, cs, base, logdet, n, batch, f.threads, s);
    default: return gj_launch_t<4, 48>(M, X, rs, cs, base, logdet, n, batch, f.threads, s);
  }
}

}  // namespace hq
