// Small kernels of the sweep: UDT bookkeeping, the end of a stabilisation
// point, block (global) moves, equal-time observables and plain copies.
#include "hq_device.h"
#include "hq_internal.h"

namespace hq {

// ---------------------------------------------------------------------------
// U = I, D = 1, T = I for every batch entry
// ---------------------------------------------------------------------------
__global__ void identity_kernel(double* U, double* D, double* T, int n) {
  const int z = blockIdx.y;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int r = e / n, q = e - r * n;
  const double v = (r == q) ? 1.0 : 0.0;
  U[(long)z * n * n + e] = v;
  T[(long)z * n * n + e] = v;
  if (q == 0) D[(long)z * n + r] = 1.0;
}

hipError_t launch_identity(double* U, double* D, double* T, int n, int batch, hipStream_t s) {
  hipLaunchKernelGGL(identity_kernel, dim3((n * n + 255) / 256, batch), dim3(256), 0, s, U, D, T, n);
  return hipGetLastError();
}

// dbinv = 1/max(D,1), ds = min(D,1); sumlog = (sumlog if accumulate) + sum log max(D,1)
__global__ void dsplit_kernel(const double* D, double* dbinv, double* ds, double* sumlog, int accumulate, int n) {
  __shared__ double red[4];
  const int z = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double d = D[(long)z * n + i];
    const double db = fmax(d, 1.0);
    dbinv[(long)z * n + i] = 1.0 / db;
    ds[(long)z * n + i] = fmin(d, 1.0);
    s += log(db);
  }
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) sumlog[z] = (accumulate ? sumlog[z] : 0.0) + s;
}

hipError_t launch_dsplit(const double* D, double* dbinv, double* ds, double* sumlog, int accumulate, int n,
                         int batch, hipStream_t s) {
  hipLaunchKernelGGL(dsplit_kernel, dim3(batch), dim3(256), 0, s, D, dbinv, ds, sumlog, accumulate, n);
  return hipGetLastError();
}

// both splits of a merge in one launch: sumlog = sum log Db_L + sum log Db_R,
// the two sums formed as the two launches of dsplit_kernel form them
__global__ void dsplit2_kernel(const double* DL, double* lbinv, double* ls, const double* DR, double* rbinv,
                               double* rs, double* sumlog, int n) {
  __shared__ double red[4];
  const int z = blockIdx.x;
  double sl = 0.0, sr = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const long e = (long)z * n + i;
    const double dl = DL[e], dr = DR[e];
    const double bl = fmax(dl, 1.0), br = fmax(dr, 1.0);
    lbinv[e] = 1.0 / bl;
    ls[e] = fmin(dl, 1.0);
    rbinv[e] = 1.0 / br;
    rs[e] = fmin(dr, 1.0);
    sl += log(bl);
    sr += log(br);
  }
  sl = block_sum<256>(sl, red);
  sr = block_sum<256>(sr, red);
  if (threadIdx.x == 0) sumlog[z] = (0.0 + sl) + sr;
}

hipError_t launch_dsplit2(const double* DL, double* lbinv, double* ls, const double* DR, double* rbinv, double* rs,
                          double* sumlog, int n, int batch, hipStream_t s) {
  hipLaunchKernelGGL(dsplit2_kernel, dim3(batch), dim3(256), 0, s, DL, lbinv, ls, DR, rbinv, rs, sumlog, n);
  return hipGetLastError();
}

// M = diag(dbinv) U^T + diag(ds) T for every chain (the merge matrix when the
// right factor is the identity), U read through 32 x 32 LDS tiles so that
// both reads and the write are row-contiguous
__global__ void merge_identity_kernel(const double* __restrict__ U, long sU, const double* __restrict__ T, long sT,
                                      const double* __restrict__ dbinv, const double* __restrict__ ds,
                                      double* __restrict__ M, int n) {
  __shared__ double tile[32][33];
  const int z = blockIdx.z;
  const int i0 = blockIdx.y * 32, j0 = blockIdx.x * 32;
  const double* u = U + (long)z * sU;
  for (int r = threadIdx.y; r < 32; r += 8) {        // tile[jj][ii] = U[j0 + jj][i0 + ii]
    const int j = j0 + r, i = i0 + threadIdx.x;
    tile[r][threadIdx.x] = (j < n && i < n) ? u[(long)j * n + i] : 0.0;
  }
  __syncthreads();
  const double* t = T + (long)z * sT;
  for (int r = threadIdx.y; r < 32; r += 8) {
    const int i = i0 + r, j = j0 + threadIdx.x;
    if (i < n && j < n) {
      const double a = dbinv[(long)z * n + i] * tile[threadIdx.x][r];
      const double b = ds[(long)z * n + i] * t[(long)i * n + j];
      M[(long)z * n * n + (long)i * n + j] = a + b;
    }
  }
}
hipError_t launch_merge_identity(const double* U, long sU, const double* T, long sT, const double* dbinv,
                                 const double* ds, double* M, int n, int batch, hipStream_t s) {
  if (n <= 0 || batch <= 0) return hipSuccess;
  const unsigned t = (unsigned)((n + 31) / 32);
  hipLaunchKernelGGL(merge_identity_kernel, dim3(t, t, batch), dim3(32, 8), 0, s, U, sU, T, sT, dbinv, ds, M, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// end of a stabilisation point: drift of the tracked G / log det against the
// FP64 recomputation, then the tracked state is replaced by it.
// drift[z] = {max |dG|, max |dlogdet|, last |dG|, last |dlogdet|, flags}
// ---------------------------------------------------------------------------
// Stabilisation finish in two launches.  The copy of the recomputed G over
// the tracked one is spread over STAB_SPLIT workgroups per chain (one per
// CU would leave most of each CU's memory pipeline idle); each writes its
// share's max |G_tracked - G_new| and non-finite flag to part[z][k].  The
// second launch folds the parts per chain and updates drift and log det.
constexpr int STAB_SPLIT = 8;

template <typename T>
__global__ __launch_bounds__(256) void stab_copy_kernel(T* G, const double* Gnew, double* part, int n, int record,
                                                        double* saved) {
  __shared__ double red[4];
  const int k = blockIdx.x, z = blockIdx.y;
  const long nn = (long)n * n;
  const long e0 = nn * k / STAB_SPLIT, e1 = nn * (k + 1) / STAB_SPLIT;
  T* g = G + z * nn;
  const double* gn = Gnew + z * nn;
  double* sv = saved ? saved + z * nn : nullptr;
  double mx = 0.0, bad = 0.0;
  batched_copy<256, 8, double>((int)(e1 - e0), [&](int e) { return gn[e0 + e]; },
                               [&](int e, double v) {
                                 if (!isfinite(v)) bad = 1.0;
                                 const double old = (double)g[e0 + e];
                                 if (record) mx = fmax(mx, fabs(old - v));
                                 if (sv) sv[e0 + e] = old;
                                 g[e0 + e] = (T)v;
                               });
  mx = block_max<256>(mx, red);
  bad = block_max<256>(bad, red);
  if (threadIdx.x == 0) {
    part[(z * STAB_SPLIT + k) * 2] = mx;
    part[(z * STAB_SPLIT + k) * 2 + 1] = bad;
  }
}

__global__ void stab_fold_kernel(const double* part, double* logdet, const double* logdet_new, double* drift,
                                 int chains, int record, double* saved_logdet) {
  const int z = blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= chains) return;
  double mx = 0.0, bad = 0.0;
  for (int k = 0; k < STAB_SPLIT; ++k) {
    mx = fmax(mx, part[(z * STAB_SPLIT + k) * 2]);
    bad = fmax(bad, part[(z * STAB_SPLIT + k) * 2 + 1]);
  }
  const double ldn = logdet_new[z];
  double* dr = drift + (long)z * 5;
  if (record) {
    const double dl = fabs(logdet[z] - ldn);
    dr[0] = fmax(dr[0], mx);
    dr[1] = fmax(dr[1], dl);
    dr[2] = mx;
    dr[3] = dl;
  }
  if (bad > 0.0 || !isfinite(ldn)) dr[4] = 1.0;
  if (saved_logdet) saved_logdet[z] = logdet[z];
  logdet[z] = ldn;
}

size_t stab_part_doubles(int batch) { return (size_t)batch * STAB_SPLIT * 2; }

hipError_t launch_stab_finish(void* G, int precision, const double* Gnew, double* logdet, const double* logdet_new,
                              double* drift, double* part, int n, int batch, int record_drift, hipStream_t s,
                              double* saved, double* saved_logdet) {
  if (batch <= 0) return hipSuccess;
  const dim3 grid(STAB_SPLIT, batch);
  if (precision)
    hipLaunchKernelGGL(stab_copy_kernel<float>, grid, dim3(256), 0, s, (float*)G, Gnew, part, n, record_drift, saved);
  else
    hipLaunchKernelGGL(stab_copy_kernel<double>, grid, dim3(256), 0, s, (double*)G, Gnew, part, n, record_drift,
                       saved);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(stab_fold_kernel, dim3((batch + 63) / 64), dim3(64), 0, s, part, logdet, logdet_new, drift,
                     batch, record_drift, saved_logdet);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// copies and fills
// ---------------------------------------------------------------------------
__global__ void f64_to_f32_kernel(float* d, const double* s, long n) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) d[e] = (float)s[e];
}
__global__ void f32_to_f64_kernel(double* d, const float* s, long n) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) d[e] = (double)s[e];
}
__global__ void copy_u32_kernel(uint32_t* d, const uint32_t* s, long n) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) d[e] = s[e];
}
__global__ void copy_f64_kernel(double* d, const double* s, long n) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) d[e] = s[e];
}
__global__ void fill_i64_kernel(int64_t* p, int64_t v, long n) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = v;
}
__global__ void fill_u8_kernel(uint8_t* p, uint8_t v, long n) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = v;
}
__global__ void fill_f64_kernel(double* p, double v, long n) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = v;
}
__global__ void add_i64_kernel(int64_t* p, int64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p += v;
}

static inline unsigned nblk(long n) { return (unsigned)((n + 255) / 256); }


// rows (the (o, i) pairs of every copy in turn) are dealt to blockIdx.y with
// stride gridDim.y
__global__ void copy_blocks_multi_kernel(BlockCopies c, long rows) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  for (long row = blockIdx.y; row < rows; row += gridDim.y) {
    long y = row;
    int q = 0;
    while (q < c.k - 1 && y >= (long)c.c[q].outer * c.c[q].inner) {
      y -= (long)c.c[q].outer * c.c[q].inner;
      ++q;
    }
    const BlockCopy& b = c.c[q];
    const long o = y / b.inner, i = y - o * b.inner;
    if (e < b.len) b.dst[o * b.dso + i * b.dsi + e] = b.src[o * b.sso + i * b.ssi + e];
  }
}
hipError_t launch_copy_blocks_multi(const BlockCopies& c, hipStream_t s) {
  BlockCopies d;
  long len = 0, rows = 0;
  for (int q = 0; q < c.k && q < 4; ++q)
    if (c.c[q].len > 0 && c.c[q].outer > 0 && c.c[q].inner > 0) {
      d.c[d.k++] = c.c[q];
      len = std::max(len, c.c[q].len);
      rows += (long)c.c[q].outer * c.c[q].inner;
    }
  if (d.k == 0) return hipSuccess;
  hipLaunchKernelGGL(copy_blocks_multi_kernel, dim3(nblk(len), (unsigned)std::min(rows, 65535L)), dim3(256), 0, s, d,
                     rows);
  return hipGetLastError();
}

hipError_t launch_copy_f64_to_f32(float* dst, const double* src, long count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3(nblk(count)), dim3(256), 0, s, dst, src, count);
  return hipGetLastError();
}
hipError_t launch_copy_u32(uint32_t* dst, const uint32_t* src, long count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_u32_kernel, dim3(nblk(count)), dim3(256), 0, s, dst, src, count);
  return hipGetLastError();
}
hipError_t launch_copy_f32_to_f64(double* dst, const float* src, long count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(f32_to_f64_kernel, dim3(nblk(count)), dim3(256), 0, s, dst, src, count);
  return hipGetLastError();
}
hipError_t launch_copy_f64(double* dst, const double* src, long count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_f64_kernel, dim3(nblk(count)), dim3(256), 0, s, dst, src, count);
  return hipGetLastError();
}
hipError_t launch_fill_i64(int64_t* p, int64_t v, long count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i64_kernel, dim3(nblk(count)), dim3(256), 0, s, p, v, count);
  return hipGetLastError();
}
hipError_t launch_fill_u8(uint8_t* p, uint8_t v, long count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u8_kernel, dim3(nblk(count)), dim3(256), 0, s, p, v, count);
  return hipGetLastError();
}
hipError_t launch_fill_f64(double* p, double v, long count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f64_kernel, dim3(nblk(count)), dim3(256), 0, s, p, v, count);
  return hipGetLastError();
}
hipError_t launch_add_i64(int64_t* p, int64_t v, hipStream_t s) {
  hipLaunchKernelGGL(add_i64_kernel, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// block (global) moves, paper section "Determinant quantum Monte Carlo":
// X_{i,l} -> X_{i,l} + d_i for every slice l.  The bosonic change is
//   dS_b = dtau [ M Omega^2 d sum_l x_{i,l} + (M Omega^2 / 2) L d^2 - g L d ]
// (the kinetic links are unchanged), the fermionic ratio needs the full
// determinant, and R = exp(2 (log|det M'| - log|det M|) - dS_b).
// ---------------------------------------------------------------------------
__global__ void global_propose_kernel(GlobalArgs a) {
  const int c = blockIdx.x;
  const int n = a.n, L = a.L;
  const int64_t sweep = *a.sweep;
  const Philox4 rn = philox4x64_10((uint64_t)(a.chain0 + c), (uint64_t)sweep, (uint64_t)a.site, KIND_GLOBAL,
                                   a.seed, 0);
  const double d = a.width * (2.0 * u53(rn.w[0]) - 1.0);
  const double* x = a.x + (long)c * L * n;
  double* xp = a.xp + (long)c * L * n;
  batched_copy<256, 16, double>(L * n, [&](int e) { return x[e]; },
                                [&](int e, double v) { xp[e] = v + ((e % n == a.site) ? d : 0.0); });
  if (threadIdx.x == 0) a.shift[c] = d;
}

hipError_t launch_global_propose(const GlobalArgs& a, int chains, hipStream_t s) {
  hipLaunchKernelGGL(global_propose_kernel, dim3(chains), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename T>
__device__ void copy_green(T* dst, const double* src, long count) {
  batched_copy<256, 16, double>((int)count, [&](int e) { return src[e]; }, [&](int e, double v) { dst[e] = (T)v; });
}

__global__ void global_accept_kernel(GlobalArgs a) {
  __shared__ double red[4];
  __shared__ int acc_s;
  const int c = blockIdx.x;
  const int n = a.n, L = a.L;
  double* x = a.x + (long)c * L * n;
  double colsum = 0.0;
  for (int l = threadIdx.x; l < L; l += blockDim.x) colsum += x[(long)l * n + a.site];
  colsum = block_sum<256>(colsum, red);
  if (threadIdx.x == 0) {
    const int64_t sweep = *a.sweep;
    const Philox4 rn = philox4x64_10((uint64_t)(a.chain0 + c), (uint64_t)sweep, (uint64_t)a.site, KIND_GLOBAL,
                                     a.seed, 0);
    const double u = u53(rn.w[1]);
    const double d = a.shift[c];
    const double g = a.g[c];
    const double mo2 = a.mass * a.omega * a.omega;
    const double ds = a.dtau * (mo2 * d * colsum + 0.5 * mo2 * L * d * d - g * L * d);
    const double lr = 2.0 * (a.logdet_new[c] - a.logdet[c]) - ds;
    const double R = exp(lr);
    int acc = (u < R) ? 1 : 0;
    const double margin = log(u) - lr;
    if (a.replay) {
      const uint8_t rp = a.replay[(long)c * n + a.site];
      if (rp != 255) {
        if (fabs(margin) <= a.band) {
          if (acc != (int)rp) a.replay_counts[2 * c] += 1;
          acc = rp;
        } else if (acc != (int)rp) {
          a.replay_counts[2 * c + 1] += 1;
        }
      }
    }
    if (a.log_margin) {
      a.log_margin[(long)c * n + a.site] = (float)margin;
      a.log_accept[(long)c * n + a.site] = (uint8_t)acc;
    }
    int64_t* cnt = a.counters + (long)c * N_COUNTERS;
    cnt[CNT_GLOBAL_P] += 1;
    cnt[CNT_GLOBAL_A] += acc;
    if (acc) a.logdet[c] = a.logdet_new[c];
    acc_s = acc;
  }
  __syncthreads();
  if (!acc_s) return;
  const double d = a.shift[c];
  for (int l = threadIdx.x; l < L; l += blockDim.x) x[(long)l * n + a.site] += d;
  const long nn = (long)n * n;
  if (a.precision)
    copy_green<float>((float*)a.G + c * nn, a.Gnew + c * nn, nn);
  else
    copy_green<double>((double*)a.G + c * nn, a.Gnew + c * nn, nn);
}

hipError_t launch_global_accept(const GlobalArgs& a, int chains, hipStream_t s) {
  hipLaunchKernelGGL(global_accept_kernel, dim3(chains), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// equal-time observables (two equal spins, Wick's theorem on G_ij = <c_i c_j^+>)
//   <n> = (2/N) sum_i (1 - G_ii),  <n_up n_dn> = (1/N) sum_i (1 - G_ii)^2,
//   S_cdw(pi,pi) = (1/N) sum_ij e_i e_j [4 (1-G_ii)(1-G_jj) + 2 (delta_ij - G_ji) G_ij],
//   <x>, <x^2> over all (l, i).
// ---------------------------------------------------------------------------
template <typename T>
__global__ void observables_kernel(ObsArgs a) {
  __shared__ double red[4];
  const int c = blockIdx.x;
  const int n = a.n, nx = a.nx;
  const T* G = (const T*)a.G + (long)c * n * n;
  double s_occ = 0.0, s_occ2 = 0.0, s_eocc = 0.0, s_pair = 0.0, bad = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double gii = (double)G[(long)i * n + i];
    const double occ = 1.0 - gii;
    const double e = (((i % nx) + (i / nx)) & 1) ? -1.0 : 1.0;
    s_occ += occ;
    s_occ2 += occ * occ;
    s_eocc += e * occ;
    s_pair += gii;
  }
  for (long e = threadIdx.x; e < (long)n * n; e += blockDim.x) {
    const int i = (int)(e / n), j = (int)(e - (long)i * n);
    const double gij = (double)G[e], gji = (double)G[(long)j * n + i];
    if (!isfinite(gij)) bad = 1.0;
    const double ei = (((i % nx) + (i / nx)) & 1) ? -1.0 : 1.0;
    const double ej = (((j % nx) + (j / nx)) & 1) ? -1.0 : 1.0;
    s_pair -= ei * ej * gji * gij;
  }
  const double* x = a.x + (long)c * a.L * n;
  double sx = 0.0, sx2 = 0.0;
  for (long e = threadIdx.x; e < (long)a.L * n; e += blockDim.x) {
    sx += x[e];
    sx2 += x[e] * x[e];
  }
  s_occ = block_sum<256>(s_occ, red);
  s_occ2 = block_sum<256>(s_occ2, red);
  s_eocc = block_sum<256>(s_eocc, red);
  s_pair = block_sum<256>(s_pair, red);
  sx = block_sum<256>(sx, red);
  sx2 = block_sum<256>(sx2, red);
  bad = block_max<256>(bad, red);
  if (threadIdx.x == 0) {
    double* o = a.out + (long)c * 5;
    o[0] = 2.0 * s_occ / n;
    o[1] = s_occ2 / n;
    o[2] = (4.0 * s_eocc * s_eocc + 2.0 * s_pair) / n;
    o[3] = sx / ((double)a.L * n);
    o[4] = sx2 / ((double)a.L * n);
    if (bad > 0.0 || !isfinite(a.logdet[c])) a.flags[c] |= 1;
  }
}

hipError_t launch_observables(const ObsArgs& a, int chains, hipStream_t s) {
  if (a.precision)
    hipLaunchKernelGGL(observables_kernel<float>, dim3(chains), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(observables_kernel<double>, dim3(chains), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace hq
