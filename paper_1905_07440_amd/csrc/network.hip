// Network-proposed local and block moves and the cumulative update (paper:
// "Local Updates", "Global Updates" and the p_c equation at its end).
//
// The fully connected network sees the displacement d and the fields of the
// 3 x 3 spatial patch over slices l-2..l+2 (45 inputs: input
// p = 9 (dl+2) + 3 (dy+1) + (dx+1), the centre p = 22 holding d), two hidden
// layers of 64 units and one linear output f.  The estimate of the move's
// fermionic change of log W is the odd part y = (f(d) - f(-d)) / 2: the move
// back (from x + d by -d, the patch unchanged) then has estimate -y, which
// makes the cumulative accept below exact.  A proposal is accepted inside the
// sweep iff u < exp(y - dS_b), the bosonic part being exact.  After the sweep
// the whole proposal is accepted with log p_c = 2 (log|det M'| - log|det M|)
// - sum y: the Metropolis-Hastings ratio of the composite move, whose reverse
// path (the same classes in the opposite order, each move undone) the sweep
// takes with the same probability because every sweep draws its direction.
//
// Visiting order: colour classes (l mod 4, iy mod 2, ix mod 2).  No two points
// of a class lie in each other's patch, so a class is one parallel launch of
// independent proposals, 16 points per wave on the matrix cores.
//
// Block moves shift a whole column x[:, i] by d.  The convolutional network
// sees three channels over l (the column, the means of the four nearest and
// of the four diagonal next-nearest neighbours' columns): a circular
// convolution along l (4 channels, kernel 4, stride 2), sigmoid, 32 dense
// sigmoid units, a linear output f; the estimate of the move's fermionic
// change is f(x_i + d) - f(x_i).  Sites go by colour classes (iy mod 2,
// ix mod 2): a site's inputs lie in its 3 x 3 neighbourhood, which holds no
// other site of its class.  n_u sweeps of local moves, then n_u of block
// moves, precede one cumulative accept.
#include "hq_device.h"
#include "hq_internal.h"

namespace hq {

__device__ inline float act(float h, int kind) {
  return kind == 0 ? fmaxf(h, 0.0f) : (h > 20.0f ? h : log1pf(expf(h)));
}

// The network on the matrix cores: each wave evaluates 16 points at a time
// with FP32 MFMA (16 x 16 x 4), the layers transposed (hidden units as the
// MFMA rows, the 16 points as its columns) so that one layer's output
// fragment is the next layer's operand in place.  Lane (r, q), r = lane & 15,
// q = lane >> 4, works on point r.
//   layer 1: H1[o][pt] = W1[o][p] In[p][pt] over the 45 inputs (padded to 48,
//            the centre input zero), MFMA step s taking p = 4 s + q, so each
//            lane gathers 12 of its point's inputs; the d-dependent term
//            W1[o][22] (+-d) and b1 are added after, once per sign.
//   layer 2: the fragment a lane holds after layer 1, hidden rows
//            16 t + 4 q + v of its point, is the B operand of step s = 4 t + v
//            when that step's k for lane group q is taken to be 16 t + 4 q + v
//            (a relabelling of the sum over the 64 hidden units); W2 is read
//            in the same labelling.
//   output:  f = W3 . act(H2 + b2) + b3, each lane summing its 16 hidden rows,
//            then across the four lane groups of the point.
// The weight fragments stay in registers for all the wave's points.
// ACT: the activation (0 ReLU, 1 softplus), fixed per instantiation.
//
// A wave takes its groups four at a time.  Lane (r, q) owns point r of the
// batch's group q: it draws that proposal's random numbers and, after the
// four evaluations, takes its accept decision, so the 64-bit generator and
// the FP64 exp/log run once per point, not once per lane of the point.
// Evaluating group k, every lane of point r reads the point's place and d
// from lane (r, k).  Decisions wait for the end of the batch, which changes
// nothing: no point of a class reads another one's field.
template <int ACT>
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
  const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;

  float w1f[4][12], w2f[4][16];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int st = 0; st < 12; ++st) {
      const int p = 4 * st + q;
      w1f[t][st] = (p < 45 && p != 22) ? W1[(16 * t + r) * 45 + p] : 0.0f;
    }
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) w2f[t][4 * u + v] = W2[(16 * t + r) * 64 + 16 * u + 4 * q + v];
  // this lane's inputs p = 4 st + q of a patch: offsets (dl + 2, dy + 1, dx + 1)
  // packed 4 bits each, and which of them exist (the centre and p >= 45 do not)
  int pof[12];
  unsigned live = 0;
#pragma unroll
  for (int st = 0; st < 12; ++st) {
    const int p = 4 * st + q;
    pof[st] = (p / 9) | (((p % 9) / 3) << 4) | ((p % 3) << 8);
    if (p < 45 && p != 22) live |= 1u << st;
  }

  const int nx = a.nx, n = a.n, L = a.L;
  const int cl = a.colour >> 2, py = (a.colour >> 1) & 1, px = a.colour & 1;
  const int hx = nx / 2, per_slice = hx * hx, nl = L / 4;
  const int per_chain = nl * per_slice;
  const long total = (long)a.chains * per_chain;
  const long groups = (total + 15) / 16;
  const long nwave = (long)gridDim.x * (blockDim.x >> 6);
  const long ln = (long)L * n;

  // the 12 inputs of the point at chain pc, slice pl, site (pix, piy)
  auto gather = [&](int pc, int pl, int pix, int piy, float (&in)[12]) {
    const double* xp = a.xp + (long)pc * ln;
#pragma unroll
    for (int st = 0; st < 12; ++st) {
      int ll = pl + (pof[st] & 15) - 2, yy = piy + ((pof[st] >> 4) & 15) - 1, xx = pix + (pof[st] >> 8) - 1;
      ll += (ll < 0) ? L : 0;
      ll -= (ll >= L) ? L : 0;
      yy += (yy < 0) ? nx : 0;
      yy -= (yy >= nx) ? nx : 0;
      xx += (xx < 0) ? nx : 0;
      xx -= (xx >= nx) ? nx : 0;
      in[st] = ((live >> st) & 1) ? (float)xp[ll * n + xx + nx * yy] : 0.0f;
    }
  };

  for (long g0 = (long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); g0 < groups; g0 += 4 * nwave) {
    // this lane's own point: point r of group g0 + q nwave (a spare lane past
    // the class repeats the last point and decides nothing)
    const long item0 = (g0 + q * nwave) * 16 + r;
    const bool valid = item0 < total;
    const long item = valid ? item0 : total - 1;
    const int c = (int)(item / per_chain);
    const int k = (int)(item - (long)c * per_chain);
    const int l = cl + 4 * (k / per_slice);
    const int rem = k % per_slice;
    const int iy = py + 2 * (rem / hx), ix = px + 2 * (rem % hx);
    const int i = ix + nx * iy;
    const long draw = (long)a.inner * ln + (long)l * n + i;
    const Philox4 rn = philox4x64_10((uint64_t)(a.chain0 + c), (uint64_t)(*a.sweep), (uint64_t)draw,
                                     KIND_NN, a.seed, 0);
    const double d = a.width * (2.0 * u53(rn.w[0]) - 1.0);
    const double u1 = u53(rn.w[1]);
    const int nk = (int)((groups - g0 + nwave - 1) / nwave) < 4 ? (int)((groups - g0 + nwave - 1) / nwave) : 4;

    float in[12], inn[12];
    gather(__shfl(c, r), __shfl(l, r), __shfl(ix, r), __shfl(iy, r), in);
    float y_own = 0.0f;
    for (int kk = 0; kk < nk; ++kk) {
      // the next group's inputs are in flight while this one is evaluated
      if (kk + 1 < nk) {
        const int src = r + 16 * (kk + 1);
        gather(__shfl(c, src), __shfl(l, src), __shfl(ix, src), __shfl(iy, src), inn);
      }
      const float df = (float)__shfl(d, r + 16 * kk);

      f4 h1[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        h1[t] = f4{0, 0, 0, 0};
#pragma unroll
        for (int st = 0; st < 12; ++st) h1[t] = mfma16(w1f[t][st], in[st], h1[t]);
      }
      float hp[4][4], hm[4][4];
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int o = 16 * t + 4 * q + v;
          const float s0 = h1[t][v] + b1[o], wd = W1[o * 45 + 22] * df;
          hp[t][v] = act(s0 + wd, ACT);
          hm[t][v] = act(s0 - wd, ACT);
        }
      f4 op[4], om[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        op[t] = f4{0, 0, 0, 0};
        om[t] = f4{0, 0, 0, 0};
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            op[t] = mfma16(w2f[t][4 * u + v], hp[u][v], op[t]);
            om[t] = mfma16(w2f[t][4 * u + v], hm[u][v], om[t]);
          }
      }
      float fp = 0.0f, fm = 0.0f;
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int o = 16 * t + 4 * q + v;
          fp = fmaf(W3[o], act(op[t][v] + b2[o], ACT), fp);
          fm = fmaf(W3[o], act(om[t][v] + b2[o], ACT), fm);
        }
      fp += __shfl_xor(fp, 16);
      fm += __shfl_xor(fm, 16);
      fp += __shfl_xor(fp, 32);
      fm += __shfl_xor(fm, 32);
      const float y = 0.5f * ((fp + b3) - (fm + b3));
      y_own = (q == kk) ? y : y_own;
#pragma unroll
      for (int st = 0; st < 12; ++st) in[st] = inn[st];
    }
    if (!valid) continue;

    double* xp = a.xp + (long)c * ln;
    const double xa = xp[(long)l * n + i];
    const double xprev = xp[(long)((l - 1 + L) % L) * n + i];
    const double xnext = xp[(long)((l + 1) % L) * n + i];
    const double g = a.g[c];
    const double kin = (a.mass / a.dtau) * (d * (2.0 * xa - xprev - xnext) + d * d);
    const double pot = a.dtau * 0.5 * a.mass * a.omega * a.omega * (2.0 * xa * d + d * d);
    const double ds = kin + pot - a.dtau * g * d;
    const double lr = (double)y_own - ds;
    int acc = (u1 < exp(lr)) ? 1 : 0;
    const double margin = log(u1) - lr;
    const long slot = (long)c * a.nu * ln + draw;       // decision log and replay
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
    const long s2 = (long)c * ln + (long)l * n + i;
    if (acc) {
      a.sum_y[s2] += (double)y_own;
      a.accepted[s2] += 1;
      xp[(long)l * n + i] = xa + d;
    }
  }
}

// one workgroup of four waves per CU; each wave takes groups of 16 points in
// turn
hipError_t launch_network_colour(const NetArgs& a, int chains, hipStream_t s) {
  const long items = (long)chains * (a.L / 4) * (a.nx / 2) * (a.nx / 2);
  const long groups = (items + 15) / 16;
  const long blocks = (groups + 3) / 4 < 256 ? (groups + 3) / 4 : 256;
  if (blocks <= 0) return hipSuccess;
  if (a.activation == 0)
    hipLaunchKernelGGL(network_colour_kernel<0>, dim3((unsigned)blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(network_colour_kernel<1>, dim3((unsigned)blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

constexpr int CNN_C = 4, CNN_K = 4, CNN_S = 2, CNN_H = 32;
size_t cnn_lds_bytes(int L) { return (size_t)(64 * L + 117) * sizeof(float); }

__device__ inline float sigm(float h) { return 1.0f / (1.0f + __expf(-h)); }

// one wave per site: the lanes take the conv positions p = lane, lane + 64,
// ... and accumulate partial dense sums for both evaluations (moved and
// unmoved column); a halving butterfly leaves the total of dense unit h of
// the unmoved evaluation in lane h and of the moved one in lane 32 + h
__global__ __launch_bounds__(256) void cnn_colour_kernel(CnnArgs a) {
  extern __shared__ float cw[];
  const int nx = a.nx, n = a.n, L = a.L, P = L / CNN_S;
  const int nw = 64 * L + 117;
  for (int e = threadIdx.x; e < nw; e += blockDim.x) cw[e] = a.w[e];
  __syncthreads();
  const float* Wc = cw;                                 // [C][3][K]
  const float* bc = Wc + CNN_C * 3 * CNN_K;             // [C]
  const float* Wd = bc + CNN_C;                         // [H][C P]
  const float* bd = Wd + CNN_H * CNN_C * P;             // [H]
  const float* Wo = bd + CNN_H;                         // [H]
  const float bo = Wo[CNN_H];

  const int lane = threadIdx.x & 63;
  const int py = (a.colour >> 1) & 1, px = a.colour & 1;
  const int hx = nx / 2, per_chain = hx * hx;
  const long item = (long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);   // one site per wave
  const int c = (int)(item / per_chain);
  if (c >= a.chains) return;                            // whole waves; no barrier follows
  const int k = (int)(item - (long)c * per_chain);
  const int iy = py + 2 * (k / hx), ix = px + 2 * (k % hx);
  const int i = ix + nx * iy;
  int nb4[4], dg4[4];
  nb4[0] = (ix + 1) % nx + nx * iy;          nb4[1] = (ix + nx - 1) % nx + nx * iy;
  nb4[2] = ix + nx * ((iy + 1) % nx);        nb4[3] = ix + nx * ((iy + nx - 1) % nx);
  dg4[0] = (ix + 1) % nx + nx * ((iy + 1) % nx);      dg4[1] = (ix + 1) % nx + nx * ((iy + nx - 1) % nx);
  dg4[2] = (ix + nx - 1) % nx + nx * ((iy + 1) % nx); dg4[3] = (ix + nx - 1) % nx + nx * ((iy + nx - 1) % nx);

  double* xp = a.xp + (long)c * L * n;
  const long draw = (long)a.inner * n + i;
  const Philox4 rn = philox4x64_10((uint64_t)(a.chain0 + c), (uint64_t)(*a.sweep), (uint64_t)draw,
                                   KIND_NN_GLOBAL, a.seed, 0);
  const double u1 = u53(rn.w[1]);
  const double d = a.width * (2.0 * u53(rn.w[0]) - 1.0);
  const float df = (float)d;
  // the moved evaluation differs only in channel 0: conv + d * sum_k Wc[c][0][k]
  float shift[CNN_C];
#pragma unroll
  for (int ch = 0; ch < CNN_C; ++ch) {
    float s = 0.0f;
#pragma unroll
    for (int kk = 0; kk < CNN_K; ++kk) s += Wc[(ch * 3 + 0) * CNN_K + kk];
    shift[ch] = df * s;
  }
  float v[2 * CNN_H];                                   // partial dense sums: unmoved, then moved
#pragma unroll
  for (int h = 0; h < 2 * CNN_H; ++h) v[h] = 0.0f;
  double colsum = 0.0;
  for (int p = lane; p < P; p += 64) {
    float in0[CNN_K], in1[CNN_K], in2[CNN_K];
#pragma unroll
    for (int kk = 0; kk < CNN_K; ++kk) {
      const int l = (CNN_S * p + kk) % L;
      const double* row = xp + (long)l * n;
      const double xi = row[i];
      if (kk < CNN_S) colsum += xi;                    // each slice once
      in0[kk] = (float)xi;
      in1[kk] = (float)(0.25 * (row[nb4[0]] + row[nb4[1]] + row[nb4[2]] + row[nb4[3]]));
      in2[kk] = (float)(0.25 * (row[dg4[0]] + row[dg4[1]] + row[dg4[2]] + row[dg4[3]]));
    }
#pragma unroll
    for (int ch = 0; ch < CNN_C; ++ch) {
      float s = bc[ch];
#pragma unroll
      for (int kk = 0; kk < CNN_K; ++kk) {
        s = fmaf(Wc[(ch * 3 + 0) * CNN_K + kk], in0[kk], s);
        s = fmaf(Wc[(ch * 3 + 1) * CNN_K + kk], in1[kk], s);
        s = fmaf(Wc[(ch * 3 + 2) * CNN_K + kk], in2[kk], s);
      }
      const float h0 = sigm(s), h1 = sigm(s + shift[ch]);
      const float* wd = Wd + ch * P + p;             // Wd[h][ch P + p], stride C P over h
#pragma unroll
      for (int h = 0; h < CNN_H; ++h) {
        const float wv = wd[(long)h * CNN_C * P];
        v[h] = fmaf(wv, h0, v[h]);
        v[CNN_H + h] = fmaf(wv, h1, v[CNN_H + h]);
      }
    }
  }
  // halving butterfly: at width w the lanes with bit w keep the upper half
#pragma unroll
  for (int w = 32; w >= 1; w >>= 1) {
    const bool up = (lane & w) != 0;
#pragma unroll
    for (int j = 0; j < w; ++j) {
      const float send = up ? v[j] : v[j + w];
      const float keep = up ? v[j + w] : v[j];
      v[j] = keep + __shfl_xor(send, w);
    }
  }
  const int h = lane & (CNN_H - 1);
  float t = Wo[h] * sigm(v[0] + bd[h]);
#pragma unroll
  for (int w = 16; w >= 1; w >>= 1) t += __shfl_xor(t, w);   // within each half of the wave
  const float f0 = bo + __shfl(t, 0), f1 = bo + __shfl(t, 32);
  const float y = f1 - f0;
#pragma unroll
  for (int w = 32; w >= 1; w >>= 1) colsum += __shfl_xor(colsum, w);

  const double g = a.g[c];
  const double mw2 = a.mass * a.omega * a.omega;
  const double ds = a.dtau * (mw2 * d * colsum + 0.5 * mw2 * L * d * d - g * L * d);
  const double lr = (double)y - ds;
  int acc = (u1 < exp(lr)) ? 1 : 0;
  const double margin = log(u1) - lr;
  const long slot = (long)c * a.nu * n + draw;
  if (a.replay) {
    const uint8_t rp = a.replay[slot];
    if (rp != 255) {
      if (fabs(margin) <= a.band) {
        if (lane == 0 && acc != (int)rp) atomicAdd((unsigned long long*)&a.replay_counts[2 * c], 1ull);
        acc = rp;
      } else if (lane == 0 && acc != (int)rp) {
        atomicAdd((unsigned long long*)&a.replay_counts[2 * c + 1], 1ull);
      }
    }
  }
  if (lane == 0) {
    if (a.log_margin) { a.log_margin[slot] = (float)margin; a.log_accept[slot] = (uint8_t)acc; }
    if (acc) {
      a.sum_y[(long)c * n + i] += (double)y;
      a.accepted[(long)c * n + i] += 1;
    }
  }
  if (acc)
    for (int l = lane; l < L; l += 64) xp[(long)l * n + i] += d;
}

hipError_t launch_cnn_colour(const CnnArgs& a, int chains, hipStream_t s) {
  if (a.L % CNN_S || cnn_lds_bytes(a.L) > 65536 || a.nx % 2) return hipErrorInvalidValue;
  const long sites = (long)chains * (a.nx / 2) * (a.nx / 2);   // one wave each, four per workgroup
  hipLaunchKernelGGL(cnn_colour_kernel, dim3((unsigned)((sites + 3) / 4)), dim3(256), cnn_lds_bytes(a.L), s, a);
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
  double sy = 0.0, na = 0.0, nbk = 0.0;
  for (long e = threadIdx.x; e < ln; e += blockDim.x) {
    sy += a.sum_y[c * ln + e];
    na += (double)a.accepted[c * ln + e];
  }
  if (a.sum_yb)
    for (long e = threadIdx.x; e < n; e += blockDim.x) {
      sy += a.sum_yb[(long)c * n + e];
      nbk += (double)a.accepted_b[(long)c * n + e];
    }
  sy = block_sum<256>(sy, red);
  na = block_sum<256>(na, red);
  nbk = block_sum<256>(nbk, red);
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
    cnt[CNT_NN_P] += (int64_t)a.inner * ln;
    cnt[CNT_NN_A] += (int64_t)na;
    if (a.sum_yb) {
      cnt[CNT_GLOBAL_P] += (int64_t)a.inner * n;
      cnt[CNT_GLOBAL_A] += (int64_t)nbk;
    }
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
}

hipError_t launch_cumulative(const CumulativeArgs& a, int chains, hipStream_t s) {
  hipLaunchKernelGGL(cumulative_kernel, dim3(chains), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace hq
