// Network-proposed local moves and the cumulative update (paper: "Local
// Updates", and the p_c equation at the end of "Global Updates").
//
// The fully connected network sees the displacement d and the fields of the
// 3 x 3 spatial patch over slices l-2..l+2 (45 inputs: input
// p = 9 (dl+2) + 3 (dy+1) + (dx+1), the centre p = 22 holding d), two hidden
// layers of 64 units and one linear output y, the estimate of the fermionic
// change of log W.  A proposal is accepted inside the sweep iff
// u < exp(y - dS_b), the bosonic part being exact.  After the sweep the whole
// proposal is accepted with log p_c = 2 (log|det M'| - log|det M|) - sum y.
//
// Visiting order: colour classes (l mod 4, iy mod 2, ix mod 2).  No two points
// of a class lie in each other's patch, so a class is one parallel launch of
// independent proposals: one thread per point, the weights in LDS.
#include "hq_device.h"
#include "hq_internal.h"

namespace hq {

__device__ inline float act(float h, int kind) {
  return kind == 0 ? fmaxf(h, 0.0f) : (h > 20.0f ? h : log1pf(expf(h)));
}

__global__ __launch_bounds__(256) void network_colour_kernel(NetArgs a) {
  __shared__ float w[7169 + 3];
  for (int e = threadIdx.x; e < 7169; e += blockDim.x) w[e] = a.w[e];
  __syncthreads();
  const float* W1 = w;
  const float* b1 = W1 + 64 * 45;
  const float* W2 = b1 + 64;
  const float* b2 = W2 + 64 * 64;
  const float* W3 = b2 + 64;
  const float b3 = W3[64];

  const int nx = a.nx, n = a.n, L = a.L;
  const int cl = a.colour >> 2, py = (a.colour >> 1) & 1, px = a.colour & 1;
  const int hx = nx / 2, per_slice = hx * hx, nl = L / 4;
  const int per_chain = nl * per_slice;
  const long item = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int c = (int)(item / per_chain);
  if (c >= a.chains) return;
  const int k = (int)(item - (long)c * per_chain);
  const int l = cl + 4 * (k / per_slice);
  const int rem = k % per_slice;
  const int iy = py + 2 * (rem / hx), ix = px + 2 * (rem % hx);
  const int i = ix + nx * iy;

  double* xp = a.xp + (long)c * L * n;
  const Philox4 rn = philox4x64_10((uint64_t)(a.chain0 + c), (uint64_t)(*a.sweep), (uint64_t)(l * n + i),
                                   KIND_NN, a.seed, 0);
  const double u1 = u53(rn.w[1]);
  const double d = a.width * (2.0 * u53(rn.w[0]) - 1.0);

  float in[45];
#pragma unroll
  for (int dl = -2; dl <= 2; ++dl) {
    const int ll = (l + dl + L) % L;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int j = (ix + dx + nx) % nx + nx * ((iy + dy + nx) % nx);
        in[9 * (dl + 2) + 3 * (dy + 1) + (dx + 1)] = (float)xp[(long)ll * n + j];
      }
  }
  in[22] = (float)d;
  float h1[64];
#pragma unroll
  for (int o = 0; o < 64; ++o) {
    float s = b1[o];
#pragma unroll
    for (int p = 0; p < 45; ++p) s = fmaf(W1[o * 45 + p], in[p], s);
    h1[o] = act(s, a.activation);
  }
  float y = b3;
#pragma unroll 4
  for (int o = 0; o < 64; ++o) {
    float s = b2[o];
#pragma unroll
    for (int p = 0; p < 64; ++p) s = fmaf(W2[o * 64 + p], h1[p], s);
    y = fmaf(W3[o], act(s, a.activation), y);
  }

  const double xa = xp[(long)l * n + i];
  const double xprev = xp[(long)((l - 1 + L) % L) * n + i];
  const double xnext = xp[(long)((l + 1) % L) * n + i];
  const double g = a.g[c];
  const double kin = (a.mass / a.dtau) * (d * (2.0 * xa - xprev - xnext) + d * d);
  const double pot = a.dtau * 0.5 * a.mass * a.omega * a.omega * (2.0 * xa * d + d * d);
  const double ds = kin + pot - a.dtau * g * d;
  const double lr = (double)y - ds;
  int acc = (u1 < exp(lr)) ? 1 : 0;
  const double margin = log(u1) - lr;
  const long slot = (long)c * L * n + (long)l * n + i;
  if (a.replay) {
    const uint8_t rp = a.replay[slot];
    if (rp != 255) {
      if (fabs(margin) <= a.band) {
        if (acc != (int)rp) atomicAdd((unsigned long long*)&a.replay_counts[2 * c], 1ull);
        acc = rp;
      } else if (acc != (int)rp) {
        atomicAdd((unsigned long long*)&a.replay_counts[2 * c + 1], 1ull);
      }
    }
  }
  if (a.log_margin) { a.log_margin[slot] = (float)margin; a.log_accept[slot] = (uint8_t)acc; }
  a.sum_y[slot] = acc ? (double)y : 0.0;
  a.accepted[slot] = (uint8_t)acc;
  if (acc) xp[(long)l * n + i] = xa + d;
}

hipError_t launch_network_colour(const NetArgs& a, int chains, hipStream_t s) {
  const long items = (long)chains * (a.L / 4) * (a.nx / 2) * (a.nx / 2);
  hipLaunchKernelGGL(network_colour_kernel, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

// one workgroup per chain: sum of accepted outputs, counters, p_c, and the
// replacement of the chain's state when the cumulative move is accepted
__global__ void cumulative_kernel(CumulativeArgs a) {
  __shared__ double red[4];
  __shared__ int acc_s;
  const int c = blockIdx.x;
  const int n = a.n, L = a.L;
  const long ln = (long)L * n;
  double sy = 0.0, na = 0.0;
  for (long e = threadIdx.x; e < ln; e += blockDim.x) {
    sy += a.sum_y[c * ln + e];
    na += (double)a.accepted[c * ln + e];
  }
  sy = block_sum<256>(sy, red);
  na = block_sum<256>(na, red);
  if (threadIdx.x == 0) {
    const Philox4 rn = philox4x64_10((uint64_t)(a.chain0 + c), (uint64_t)(*a.sweep), 0, KIND_CUMULATIVE,
                                     a.seed, 0);
    const double u = u53(rn.w[0]);
    const double lpc = 2.0 * (a.logdet_new[c] - a.logdet[c]) - sy;
    int acc = (u < exp(lpc)) ? 1 : 0;
    const double margin = log(u) - lpc;
    if (a.replay) {
      const uint8_t rp = a.replay[c];
      if (rp != 255) {
        if (fabs(margin) <= a.band) {
          if (acc != (int)rp) a.replay_counts[2 * c] += 1;
          acc = rp;
        } else if (acc != (int)rp) {
          a.replay_counts[2 * c + 1] += 1;
        }
      }
    }
    if (a.log_margin) { a.log_margin[c] = (float)margin; a.log_accept[c] = (uint8_t)acc; }
    int64_t* cnt = a.counters + (long)c * N_COUNTERS;
    cnt[CNT_NN_P] += ln;
    cnt[CNT_NN_A] += (int64_t)na;
    cnt[CNT_CUM_P] += 1;
    cnt[CNT_CUM_A] += acc;
    a.last_log_pc[2 * c] = lpc;
    a.last_log_pc[2 * c + 1] = sy;
    if (acc) a.logdet[c] = a.logdet_new[c];
    acc_s = acc;
  }
  __syncthreads();
  if (!acc_s) return;
  double* x = a.x + c * ln;
  const double* xp = a.xp + c * ln;
  batched_copy<256, 16, double>((int)ln, [&](int e) { return xp[e]; }, [&](int e, double v) { x[e] = v; });
  const long nn = (long)n * n;
  const double* gn = a.Gnew + c * nn;
  if (a.precision) {
    float* G = (float*)a.G + c * nn;
    batched_copy<256, 16, double>((int)nn, [&](int e) { return gn[e]; }, [&](int e, double v) { G[e] = (float)v; });
  } else {
    double* G = (double*)a.G + c * nn;
    batched_copy<256, 16, double>((int)nn, [&](int e) { return gn[e]; }, [&](int e, double v) { G[e] = v; });
  }
  const long nbk = (long)a.nb * nn;
  const double* bp = a.blkp + c * nbk;
  double* bk = a.blk + c * nbk;
  batched_copy<256, 16, double>((int)nbk, [&](int e) { return bp[e]; }, [&](int e, double v) { bk[e] = v; });
}

hipError_t launch_cumulative(const CumulativeArgs& a, int chains, hipStream_t s) {
  hipLaunchKernelGGL(cumulative_kernel, dim3(chains), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace hq
