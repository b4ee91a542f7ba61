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
// Delayed form: after p accepted moves at sites i_1..i_p,
//     G_cur = G0 - A Bv^T,  A[:,m] = c_m G_{m-1}[:,i_m],  Bv[:,m] = e_{i_m} - G_{m-1}[i_m,:]^T
// with c_m = delta_m / r_m.  Row by row this is a short recurrence:
//     A[j,m]  = c_m (G0[j,i_m] - sum_{m'<m} A[j,m'] Bv[i_m,m'])
//     Bv[j,m] = [j = i_m] - G0[i_m,j] + sum_{m'<m} A[i_m,m'] Bv[j,m']
// and G0 <- G0 - A Bv^T is one rank-p MFMA product.
//
// Design (submatrix blocks): the sites are taken K at a time.  For a block S
// of K consecutive sites the decisions need only G_cur[S,S], so one "walker"
// wave holds that K x K block in registers (K*K/64 entries per lane), takes
// the K decisions in order with no barrier, and applies each accepted rank-1
// update to the block alone (one shuffle and one FMA per entry).  The walker
// also records A[S,m] and Bv[S,m], the only entries the row recurrences above
// need from other rows.  Then all four waves run the recurrences for every
// row of A and Bv (the rows are independent) and apply the rank-p flush, and
// the next block starts from the flushed G.  The result is the sequential
// rank-1 chain up to rounding order.
//
// Two forms of the same slice:
//   local_regs_kernel    G lives in the MFMA accumulators of the four waves
//                        for the whole slice (the register file is larger than
//                        LDS); only the K columns and K rows of the current
//                        block pass through LDS.  The flush is pure MFMA work.
//   local_stream_kernel  G stays in global memory and the flush streams it in
//                        batches of tiles: any N <= 256, any K.
#include <type_traits>

#include "hq_device.h"
#include "hq_internal.h"

namespace hq {

__host__ __device__ inline int pad16(int n) { return (n + 15) / 16 * 16; }
__host__ __device__ inline int pad64(int n) { return (n + 63) / 64 * 64; }
__host__ __device__ inline size_t align16(size_t b) { return (b + 15) / 16 * 16; }

// per-site constants of the slice: delta, exp(-dS_b), u and the displacement
struct SiteConst { double delta, bos, u, d; };

// the accepted moves of the current block
struct BlockHdr {
  int p[2];
  int site[32];
  double c[32];
};

__device__ inline int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ inline float bcast(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ inline double bcast(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}
// the value v of lane src, src chosen per lane
__device__ inline float from_lane(float v, int src) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}
__device__ inline double from_lane(double v, int src) {
  const int lo = __builtin_amdgcn_ds_bpermute(src << 2, __double2loint(v));
  const int hi = __builtin_amdgcn_ds_bpermute(src << 2, __double2hiint(v));
  return __hiloint2double(hi, lo);
}

struct WalkState {
  double logr;
  int nacc;
  int counts[2];   // replay overrides inside the band, disagreements outside it
};

// Site constants of the slice for sites j = tid, tid + 256, ... (they do not
// depend on G); replay bits into rp[], accept flags cleared.
__device__ inline void site_constants(const LocalArgs& a, int c, SiteConst* sc, uint8_t* rp, uint8_t* flags,
                                      double* Rv) {
  const int n = a.n, L = a.L, s = a.slice;
  const double* x = a.x + (long)c * L * n;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const int64_t sweep = *a.sweep;
    const double gc = a.g[c];
    const double xa = x[s * n + j];
    const double xprev = x[((s - 1 + L) % L) * n + j];
    const double xnext = x[((s + 1) % L) * n + j];
    const Philox4 rn = philox4x64_10((uint64_t)(a.chain0 + c), (uint64_t)sweep, (uint64_t)(s * n + j), KIND_LOCAL,
                                     a.seed, 0);
    const double d = a.width * (2.0 * u53(rn.w[0]) - 1.0);
    const double kin = (a.mass / a.dtau) * (d * (2.0 * xa - xprev - xnext) + d * d);
    const double pot = a.dtau * 0.5 * a.mass * a.omega * a.omega * (2.0 * xa * d + d * d);
    SiteConst k;
    k.delta = expm1(-a.dtau * gc * d);
    k.bos = exp(-(kin + pot - a.dtau * gc * d));
    k.u = u53(rn.w[1]);
    k.d = d;
    sc[j] = k;
    rp[j] = a.replay ? a.replay[(long)c * L * n + s * n + j] : (uint8_t)255;
    flags[j] = 0;
    Rv[j] = 1.0;
  }
}

// The walker (one wave): the decisions of the block of cnt <= K sites
// starting at `base`, on G_cur[S,S] = gget(r, c) held in registers.
// Records the accepted sites and c_m in hdr, A[S,m] in As[m][.] and Bv[S,m]
// in Bs[m][.].
template <typename T, int K, typename GetG>
__device__ inline void walk_block(GetG gget, int base, int cnt, int blk, const SiteConst* sc, const uint8_t* rp,
                                  BlockHdr* hdr, T* As, T* Bs, uint8_t* flags, double* Rv, bool test_hooks,
                                  double band_lo, double band_hi, WalkState& st) {
  constexpr int RPV = K * K / 64;          // block rows per lane
  const int lane = threadIdx.x & 63;
  const int col = lane % K, rb = lane / K;
  T gs[RPV];
#pragma unroll
  for (int v = 0; v < RPV; ++v) {
    const int r = rb * RPV + v;
    gs[v] = (r < cnt && col < cnt) ? gget(r, col) : T(0);
  }
  SiteConst my = {0.0, 0.0, 2.0, 0.0};
  int my_rp = 255;
  if (lane < cnt) {
    my = sc[base + lane];
    my_rp = rp[base + lane];
  }
  double lp = 1.0;                         // product of |r| over the accepted moves
  int m = 0;
#pragma unroll
  for (int q = 0; q < K; ++q) {
    if (q < cnt) {                         // a guard, not a break: the loop stays unrolled
      const double dg = (double)bcast(gs[q % RPV], q + K * (q / RPV));
      const double delta = bcast(my.delta, q);
      const double r = 1.0 + delta * (1.0 - dg);
      const double R = r * r * bcast(my.bos, q);
      const double u = bcast(my.u, q);
      int acc = (u < R) ? 1 : 0;
      if (test_hooks) {
        // replay inside the tie band |ln u - ln R| <= band, tested as
        // R e^-band <= u <= R e^band; ln u - ln R is formed after the walk
        const int rpi = __builtin_amdgcn_readlane(my_rp, q);
        if (rpi != 255) {
          if (u >= R * band_lo && u <= R * band_hi) {
            st.counts[0] += (acc != rpi) ? 1 : 0;
            acc = rpi;
          } else {
            st.counts[1] += (acc != rpi) ? 1 : 0;
          }
        }
        if (lane == 0) Rv[base + q] = R;
      }
      acc = uniform(acc);                  // a scalar branch: every lane holds the same value
      if (acc) {
        // rank-1 update of the block; column m of A and Bv on the rows of S
        const T coef = (T)(delta / r);
        T colv[RPV];
#pragma unroll
        for (int v = 0; v < RPV; ++v) colv[v] = from_lane(gs[v], q + K * rb);
        const T rowv = from_lane(gs[q % RPV], col + K * (q / RPV));
        const T nb = ((col == q) ? T(1) : T(0)) - rowv;
        if (col == q) {
#pragma unroll
          for (int v = 0; v < RPV; ++v) As[m * K + rb * RPV + v] = coef * gs[v];
        }
        if (rb == q / RPV) Bs[m * K + col] = nb;
#pragma unroll
        for (int v = 0; v < RPV; ++v) gs[v] -= (coef * colv[v]) * nb;
        if (lane == 0) {
          hdr->site[m] = base + q;
          hdr->c[m] = delta / r;
          flags[base + q] = 1;
        }
        lp *= fabs(r);
        m = uniform(m + 1);
      }
    }
  }
  st.logr += log(lp);
  st.nacc += m;
  if (lane == 0) hdr->p[blk & 1] = m;
}

// A and Bv at the accepted rows, for the recurrences:
//   ASm[m][m'] = A[i_m, m'], BSm[m][m'] = Bv[i_m, m'] for m' < m < p, else 0
template <typename T, int K>
__device__ inline void gather_small(const BlockHdr* hdr, const T* As, const T* Bs, T* ASm, T* BSm, int base, int p) {
  for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
    const int mi = e / K, mj = e - mi * K;
    T av = T(0), bv = T(0);
    if (mi < p && mj < mi) {
      const int li = hdr->site[mi] - base;
      av = As[mj * K + li];
      bv = Bs[mj * K + li];
    }
    ASm[e] = av;
    BSm[e] = bv;
  }
}

// One row of the recurrences over KE >= p steps (entries >= p come out 0).
//   A row (isA):  v[m] = c_m (g[m] - sum_{m'<m} v[m'] BSm[m][m'])     g[m] = G0[j, i_m]
//   Bv row:       v[m] = [j = i_m] - g[m] + sum_{m'<m} ASm[m][m'] v[m']  g[m] = G0[i_m, j]
// The step constants (i_m, c_m) are read per step as wave-uniform values so
// that they sit in scalar registers.
__device__ inline int uniform_site(const BlockHdr* hdr, int mq, int p) { return uniform(hdr->site[min(mq, p - 1)]); }
__device__ inline double uniform_c(const BlockHdr* hdr, int mq, int p) {
  const double c = hdr->c[min(mq, p - 1)];
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(c));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(c));
  return __hiloint2double(hi, lo);
}

__device__ inline float uniform_val(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ inline double uniform_val(double v) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

// isA and W are the same for every lane of the wave: the W entries then live
// in scalar registers instead of one vector register each
template <typename T, int K, int KE>
__device__ inline void recur_row(const BlockHdr* hdr, int p, bool isA, bool live, int j, const T (&g)[KE],
                                 const T* W, T (&v)[KE]) {
  const T sg = isA ? T(-1) : T(1);
#pragma unroll
  for (int mq = 0; mq < KE; ++mq) {
    const int im = uniform_site(hdr, mq, p);
    T a0 = isA ? g[mq] : (((j == im) ? T(1) : T(0)) - g[mq]);
    T a1 = T(0);
#pragma unroll
    for (int m2 = 0; m2 < mq; ++m2) {
      const T w = uniform_val(W[mq * K + m2]);
      if (m2 & 1) a1 += v[m2] * w;
      else a0 += sg * (v[m2] * w);
    }
    const T mul = (mq < p) ? (isA ? (T)uniform_c(hdr, mq, p) : T(1)) : T(0);
    v[mq] = live ? mul * (a0 + sg * a1) : T(0);
  }
}

// ===========================================================================
// register-resident form
// ===========================================================================
// Four waves, one per SIMD, so that each has the whole register file of its
// SIMD.  They hold G in their MFMA accumulators for the whole slice, as a
// 2 x 2 grid over the nt x nt tiles: wave (wr, wc) = (w & 1, w >> 1) holds
// tiles (wr + 2a, wc + 2b), so every tile address of a wave is one base plus
// a compile-time offset.  Per block of K sites:
//   walk     wave 0 takes the K decisions on the K x K block G_cur[S, S]
//            (walk_diag below) and records A[S, m], Bv[S, m], i_m and c_m;
//   rows     every thread runs the row recurrences for one row j of A and
//            of Bv, reading G0[j, i_m] and G0[i_m, j] from the strips;
//   flush    the tile waves apply G -= A Bv^T on the accumulators (MFMA)
//            and extract the next block's strips G[:, S'] and G[S', :].
// Three barriers per block.
//
// LDS (bytes): header | site constants | replay bits | flags | ratios R |
// A, Bv panels [P][KL] | Cs = G[:, S] [P][K+1] | Rs = G[S, :] [K][P+1] |
// records A[S, m], Bv[S, m] [K][KR] each.  P = 32 H rows, H = (NT + 1) / 2:
// every tile row of every wave's 2 x 2 grid, those past N included (zero).
template <typename T, int K, int NT>
struct RegLds {
  enum { KL = K + 16 / (int)sizeof(T), KR = K + 16 / (int)sizeof(T), P = 32 * ((NT + 1) / 2) };
  static __host__ __device__ size_t sc() { return align16(sizeof(BlockHdr)); }
  static __host__ __device__ size_t rp(int n) { return sc() + sizeof(SiteConst) * (size_t)n; }
  static __host__ __device__ size_t flags(int n) { return rp(n) + n; }
  static __host__ __device__ size_t rv(int n) { return align16(flags(n) + n); }
  static __host__ __device__ size_t ap(int n) { return align16(rv(n) + 8 * (size_t)n); }
  static __host__ __device__ size_t bp(int n) { return ap(n) + sizeof(T) * (size_t)P * KL; }
  static __host__ __device__ size_t cs(int n) { return bp(n) + sizeof(T) * (size_t)P * KL; }
  static __host__ __device__ size_t rs(int n) { return cs(n) + sizeof(T) * (size_t)P * (K + 1); }
  static __host__ __device__ size_t ar(int n) { return align16(rs(n) + sizeof(T) * (size_t)K * (P + 1)); }
  static __host__ __device__ size_t br(int n) { return ar(n) + sizeof(T) * (size_t)K * KR; }
  static __host__ __device__ size_t total(int n) { return align16(br(n) + sizeof(T) * (size_t)K * KR); }
};

template <typename T, int NT>
struct RegTiles {
  enum { H = (NT + 1) / 2 };
  typename Frag<T>::type t[H][H];
};

// an opaque copy of v: address arithmetic derived from it is not merged with
// earlier arithmetic on v, so those addresses need not stay live in registers
__device__ inline int opaque(int v) {
  asm volatile("" : "+s"(v));
  return v;
}

// 1/r to a few ulp: the hardware seed and two Newton steps
__device__ inline double recip(double r) {
  double y = __builtin_amdgcn_rcp(r);
  y = fma(fma(-r, y, 1.0), y, y);
  return fma(fma(-r, y, 1.0), y, y);
}
__device__ inline float recip(float r) { return __builtin_amdgcn_rcpf(r); }

// The thresholds of a site's Metropolis test on G_kk (walk_diag explains them)
template <typename T>
__device__ inline void site_thresholds(const SiteConst& my, T& ksg, T& kthr, T& kthr2) {
  const double sq = sqrt(my.u / my.bos);
  if (my.delta > 0.0) {
    kthr = (T)(1.0 - (sq - 1.0) / my.delta);
    kthr2 = (T)(1.0 + (1.0 + sq) / my.delta);
  } else if (my.delta < 0.0) {
    ksg = T(-1);
    kthr = (T)(-(1.0 - (sq - 1.0) / my.delta));
    kthr2 = (T)(-(1.0 + (1.0 + sq) / my.delta));
  } else {
    kthr = (my.u < my.bos) ? (T)INFINITY : (T)-INFINITY;
    kthr2 = (T)INFINITY;
  }
}

// The walker: the decisions of the block of cnt <= K sites at `base` on
// G_cur[S, S] (g0(r, c) = G0[base + r][base + c]).
//
// Lane k (mod K) owns site base + k: it holds row k and column k of the
// block and its diagonal entry d_k, and keeps its own ratio
//     r_k = 1 + delta_k (1 - d_k),  R_k = r_k^2 exp(-dS_b,k),  accept_k = u_k < R_k
// current, so the decision on site q is bit q of one ballot.  An accepted
// move at q with c = delta_q / r_q changes the rest of the block by
//     G'[a][b] = G[a][b] + c G[a][q] G[q][b]        (a, b != q)
// so the diagonal of lane k moves by c G[k][q] G[q][k], two values lane k
// holds: the ratios of the remaining sites are new after one multiply-add
// per lane.  The rows and columns are then brought up to date with lane q's
// row and column, broadcast one entry at a time (only entries after q are
// read again).  The lane also records A[k, m] = c G[k][q] and
// Bv[k, m] = [k = q] - G[q][k], the entries of the accepted moves' rank-1
// factors on the block rows, which the row recurrences need.
template <typename T, int K, bool HOOKS, typename GetG>
__device__ __attribute__((always_inline)) inline void walk_diag(GetG g0, int base, int cnt, int blk,
                                                                const SiteConst* sc, const uint8_t* rp, BlockHdr* hdr,
                                                                T* Arec, T* Brec, uint8_t* flags, double* Rv,
                                                                double band_lo, double band_hi, WalkState& st) {
  constexpr int KR = K + 16 / (int)sizeof(T);
  const int lane = threadIdx.x & 63;
  const int k = lane & (K - 1);
  const bool act = k < cnt;
  T row[K], col[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    row[j] = (act && j < cnt) ? g0(k, j) : T(0);
    col[j] = (act && j < cnt) ? g0(j, k) : T(0);
  }
  T dg = act ? g0(k, k) : T(0);
  SiteConst my = {0.0, 0.0, 2.0, 0.0};     // u = 2: never accepted
  int my_rp = 255;
  if (act) {
    my = sc[base + k];
    my_rp = rp[base + k];
  }
  // The Metropolis test u < R = r^2 exp(-dS_b), r = 1 + delta (1 - G_kk), as
  // a test on G_kk alone: u < R is |r| > s = sqrt(u exp(dS_b)), i.e. r > s or
  // r < -s.  With sg = sign(delta), r > s is sg G_kk < kthr,
  // kthr = sg (1 - (s - 1) / delta), and r < -s is sg G_kk > kthr2,
  // kthr2 = sg (1 + (1 + s) / delta) (a determinant ratio of either sign: far
  // outside the range of G_kk at the local moves' widths, but kept so that
  // the test is the stated one).  Both are set once per block.  (delta = 0:
  // r = 1, the test is u < exp(-dS_b) whatever G_kk.)
  T ksg = T(1), kthr, kthr2;
  site_thresholds(my, ksg, kthr, kthr2);
  T gacc = T(0);                           // this lane's G_kk when its own move was accepted
  bool mine = false;
  T coef = T(0);
  double R = 0.0;
  int nover = 0, nmis = 0;
  // this lane's decision on the current diagonal (the replayed bit inside the
  // band in the test build) and its coefficient c = delta / r in case it is
  // accepted
  auto judge = [&]() -> bool {
    bool a = (ksg * dg < kthr) || (ksg * dg > kthr2);
    const T rt = fma((T)my.delta, T(1) - dg, T(1));
    coef = (T)my.delta * recip(rt);
    if (HOOKS) {
      const double r = 1.0 + my.delta * (1.0 - (double)dg);
      R = r * r * my.bos;
      if (my_rp != 255 && my.u >= R * band_lo && my.u <= R * band_hi) a = my_rp != 0;
    }
    return a;
  };
  uint64_t ball = __ballot(judge());
  int m = 0;
#pragma unroll
  for (int q = 0; q < K; ++q) {
    if (q < cnt) {                         // a guard, not a break: the loop stays unrolled
      if (HOOKS && lane == q) {
        // the site's own ratio at its decision: logged, and the replay counted
        Rv[base + q] = R;
        if (my_rp != 255) {
          const int raw = ((ksg * dg < kthr) || (ksg * dg > kthr2)) ? 1 : 0;
          if (my.u >= R * band_lo && my.u <= R * band_hi) nover += (raw != my_rp) ? 1 : 0;
          else nmis += (raw != my_rp) ? 1 : 0;
        }
      }
      if ((ball >> q) & 1) {               // a scalar branch on the ballot bit
        const T c = bcast(coef, q);
        const bool self = k == q;
        const T gkq = self ? dg : row[q];  // G[k][q]
        const T gqk = self ? dg : col[q];  // G[q][k]
        const T ak = c * gkq;              // A[k, m]
        gacc = self ? dg : gacc;
        mine = mine || self;
        dg = dg + ak * gqk;                // the diagonal first: the next decision waits on it
        ball = __ballot(judge());
        if (lane < K) {
          Arec[k * KR + m] = ak;
          Brec[k * KR + m] = (self ? T(1) : T(0)) - gqk;
        }
        const T cg = c * gqk;
#pragma unroll
        for (int j = q + 1; j < K; ++j) {
          const T rqj = bcast(row[j], q);  // G[q][j]
          const T cjq = bcast(col[j], q);  // G[j][q]
          row[j] += ak * rqj;
          col[j] += cg * cjq;
        }
        if (lane == 0) {
          hdr->site[m] = base + q;
          hdr->c[m] = (double)c;
          flags[base + q] = 1;
        }
        m = uniform(m + 1);
      }
    }
  }
  // log|r| of the accepted moves (r in FP64 from the diagonal at acceptance)
  // and the replay counts, over the owning lanes
  double lr = (lane < K && mine) ? log(fabs(1.0 + my.delta * (1.0 - (double)gacc))) : 0.0;
  lr = wave_sum(lr);
  st.logr += lr;
  if (HOOKS) {
    st.counts[0] += wave_sum(lane < K ? nover : 0);
    st.counts[1] += wave_sum(lane < K ? nmis : 0);
  }
  st.nacc += m;
  if (lane == 0) hdr->p[blk & 1] = m;
}

// The same walk for blocks of 16 sites with all 64 lanes at work.  Lane
// k + 16 g (k < 16, g < 4) holds, for s < 4, the entries G[k][4s + g] and
// G[4s + g][k] of the block, and every row of 16 lanes keeps a copy of the
// diagonal and of the sites' constants.  The update after an accepted move at
// q touches G[k][j] with G[q][j] and G[j][k] with G[j][q]: both are held by
// lane q of the same 16-lane row, so one row broadcast (DPP row_newbcast)
// serves the four row groups at once, 4 entries per lane instead of 16.  The
// two coefficients G[k][q] and G[q][k] live in row group q mod 4 and reach the
// others through two lane-swap steps (v_permlane16_swap, v_permlane32_swap).
template <int Q> __device__ inline float row_bcast(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x150 + Q, 0xF, 0xF, true));
}
template <int Q> __device__ inline double row_bcast(double v) {
  return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + Q, 0xF, 0xF, true);
}
// the value row group G holds, in every row group
template <int G> __device__ inline unsigned from_group(unsigned v) {
  const auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);   // [r0 r0 r2 r2], [r1 r1 r3 r3]
  const unsigned z = (G & 1) ? p[1] : p[0];
  const auto w = __builtin_amdgcn_permlane32_swap(z, z, false, false);   // [z0 z1 z0 z1], [z2 z3 z2 z3]
  return (G >> 1) ? w[1] : w[0];
}
template <int G> __device__ inline float from_group(float v) { return __uint_as_float(from_group<G>(__float_as_uint(v))); }
template <int G> __device__ inline double from_group(double v) {
  const unsigned lo = from_group<G>((unsigned)__double2loint(v)), hi = from_group<G>((unsigned)__double2hiint(v));
  return __hiloint2double((int)hi, (int)lo);
}

template <typename T, bool HOOKS, typename GetG>
__device__ __attribute__((always_inline)) inline void walk_dense(GetG g0, int base, int cnt, int blk,
                                                                 const SiteConst* sc, const uint8_t* rp, BlockHdr* hdr,
                                                                 T* Arec, T* Brec, uint8_t* flags, double* Rv,
                                                                 double band_lo, double band_hi, WalkState& st) {
  constexpr int K = 16, KR = K + 16 / (int)sizeof(T);
  const int lane = threadIdx.x & 63;
  const int k = lane & 15, grp = lane >> 4;
  const bool act = k < cnt;
  T R[4], C[4];                            // R[s] = G[k][4s + grp], C[s] = G[4s + grp][k]
#pragma unroll
  for (int s4 = 0; s4 < 4; ++s4) {
    const int j = 4 * s4 + grp;
    R[s4] = (act && j < cnt) ? g0(k, j) : T(0);
    C[s4] = (act && j < cnt) ? g0(j, k) : T(0);
  }
  T dg = act ? g0(k, k) : T(0);
  SiteConst my = {0.0, 0.0, 2.0, 0.0};     // u = 2: never accepted
  int my_rp = 255;
  if (act) {
    my = sc[base + k];
    my_rp = rp[base + k];
  }
  // the Metropolis test as a test on G_kk (see walk_diag)
  T ksg = T(1), kthr, kthr2;                 // the threshold test of walk_diag
  site_thresholds(my, ksg, kthr, kthr2);
  T gacc = T(0);
  bool mine = false;
  T coef = T(0);
  double Rr = 0.0;
  int nover = 0, nmis = 0;
  auto judge = [&]() -> bool {
    bool a = (ksg * dg < kthr) || (ksg * dg > kthr2);
    const T rt = fma((T)my.delta, T(1) - dg, T(1));
    coef = (T)my.delta * recip(rt);
    if (HOOKS) {
      const double r = 1.0 + my.delta * (1.0 - (double)dg);
      Rr = r * r * my.bos;
      if (my_rp != 255 && my.u >= Rr * band_lo && my.u <= Rr * band_hi) a = my_rp != 0;
    }
    return a;
  };
  uint64_t ball = __ballot(judge());
  int m = 0;
  auto step = [&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr int qs = q >> 2, qg = q & 3;
    if (q >= cnt) return;
    if (HOOKS && lane == q) {
      Rv[base + q] = Rr;
      if (my_rp != 255) {
        const int raw = ((ksg * dg < kthr) || (ksg * dg > kthr2)) ? 1 : 0;
        if (my.u >= Rr * band_lo && my.u <= Rr * band_hi) nover += (raw != my_rp) ? 1 : 0;
        else nmis += (raw != my_rp) ? 1 : 0;
      }
    }
    if ((ball >> q) & 1) {                 // a scalar branch on the ballot bit
      const T c = bcast(coef, q);
      const bool self = k == q;
      const T gkq = self ? dg : from_group<qg>(R[qs]);   // G[k][q]
      const T gqk = self ? dg : from_group<qg>(C[qs]);   // G[q][k]
      const T ak = c * gkq;                // A[k, m]
      gacc = self ? dg : gacc;
      mine = mine || self;
      dg = dg + ak * gqk;
      ball = __ballot(judge());
      if (lane < K) {
        Arec[k * KR + m] = ak;
        Brec[k * KR + m] = (self ? T(1) : T(0)) - gqk;
      }
      const T cg = c * gqk;
#pragma unroll
      for (int s4 = qs; s4 < 4; ++s4) {    // entries j = 4 s4 + grp; those with j <= q are not read again
        R[s4] += ak * row_bcast<q>(R[s4]);   // G[k][j] += c G[k][q] G[q][j]
        C[s4] += cg * row_bcast<q>(C[s4]);   // G[j][k] += c G[q][k] G[j][q]
      }
      if (lane == 0) {
        hdr->site[m] = base + q;
        hdr->c[m] = (double)c;
        flags[base + q] = 1;
      }
      m = uniform(m + 1);
    }
  };
  step(std::integral_constant<int, 0>());
  step(std::integral_constant<int, 1>());
  step(std::integral_constant<int, 2>());
  step(std::integral_constant<int, 3>());
  step(std::integral_constant<int, 4>());
  step(std::integral_constant<int, 5>());
  step(std::integral_constant<int, 6>());
  step(std::integral_constant<int, 7>());
  step(std::integral_constant<int, 8>());
  step(std::integral_constant<int, 9>());
  step(std::integral_constant<int, 10>());
  step(std::integral_constant<int, 11>());
  step(std::integral_constant<int, 12>());
  step(std::integral_constant<int, 13>());
  step(std::integral_constant<int, 14>());
  step(std::integral_constant<int, 15>());
  double lr = (lane < K && mine) ? log(fabs(1.0 + my.delta * (1.0 - (double)gacc))) : 0.0;
  lr = wave_sum(lr);
  st.logr += lr;
  if (HOOKS) {
    st.counts[0] += wave_sum(lane < K ? nover : 0);
    st.counts[1] += wave_sum(lane < K ? nmis : 0);
  }
  st.nacc += m;
  if (lane == 0) hdr->p[blk & 1] = m;
}

// Rows of A and Bv for the flush, one row j per thread over `rows` rows
// (rows >= n come out zero), KE >= p steps:
//   A[j, m]  = c_m (G0[j, i_m] - sum_{m'<m} A[j, m'] Bv[i_m, m'])
//   Bv[j, m] = [j = i_m] - G0[i_m, j] + sum_{m'<m} A[i_m, m'] Bv[j, m']
// G0[j, i_m] = Cs[j][i_m - base], G0[i_m, j] = Rs[i_m - base][j]; A[i_m, .]
// and Bv[i_m, .] are the walker's records of row i_m - base.  Entries m >= p
// are zero.  The inputs of step m + 1 are loaded while step m computes, and a
// scheduling barrier keeps later steps' loads from being hoisted (all of them
// in flight at once would not fit the registers next to the tiles of G).
template <typename T, int K, int KE>
__device__ __attribute__((always_inline)) inline void recur_rows(const BlockHdr* hdr, int p, int base, int n, int rows,
                                                                 const T* Cs, int cl, const T* Rs, int rl,
                                                                 const T* Arec, const T* Brec, T* Ap, T* Bp) {
  constexpr int KR = K + 16 / (int)sizeof(T), KL = K + 16 / (int)sizeof(T);
  for (int j = threadIdx.x; j < rows; j += blockDim.x) {
    const bool live = j < n;
    T a[KE], b[KE];
    T wa[2][KE], wb[2][KE], ga[2], gb[2], cm[2];
    int im[2];
    auto fetch = [&](int mq, int slot) {
      const int mc = min(mq, p - 1);
      im[slot] = hdr->site[mc] - base;
      cm[slot] = (T)hdr->c[mc];
      ga[slot] = live ? Cs[j * cl + im[slot]] : T(0);
      gb[slot] = live ? Rs[im[slot] * rl + j] : T(0);
      // Bv[i_m, m'] and A[i_m, m'] for m' < m, 16 bytes at a time (the record
      // rows are 16-byte aligned and K + 16 / sizeof(T) long)
      constexpr int V = 16 / (int)sizeof(T);
      typedef T vec __attribute__((ext_vector_type(V)));
      const vec* vb = (const vec*)(Brec + im[slot] * KR);
      const vec* va = (const vec*)(Arec + im[slot] * KR);
#pragma unroll
      for (int g = 0; g < (KE + V - 1) / V; ++g) {
        if (g * V < mq) {
          const vec b4 = vb[g], a4 = va[g];
#pragma unroll
          for (int e = 0; e < V; ++e) {
            if (g * V + e < KE) {
              wb[slot][g * V + e] = b4[e];
              wa[slot][g * V + e] = a4[e];
            }
          }
        }
      }
    };
    fetch(0, 0);
#pragma unroll
    for (int mq = 0; mq < KE; ++mq) {
      const int cur = mq & 1;
      if (mq + 1 < KE) fetch(mq + 1, cur ^ 1);
      T sa = ga[cur];
      T sb = ((j == base + im[cur]) ? T(1) : T(0)) - gb[cur];
      T sa1 = T(0), sb1 = T(0);
#pragma unroll
      for (int m2 = 0; m2 < mq; ++m2) {
        if (m2 & 1) {
          sa1 -= a[m2] * wb[cur][m2];
          sb1 += wa[cur][m2] * b[m2];
        } else {
          sa -= a[m2] * wb[cur][m2];
          sb += wa[cur][m2] * b[m2];
        }
      }
      a[mq] = (mq < p) ? cm[cur] * (sa + sa1) : T(0);
      b[mq] = (mq < p) ? sb + sb1 : T(0);
      Ap[j * KL + mq] = a[mq];
      Bp[j * KL + mq] = b[mq];
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int mq = KE; mq < ((KE + 3) & ~3); ++mq) {   // zero columns up to the flush's group of four
      Ap[j * KL + mq] = T(0);
      Bp[j * KL + mq] = T(0);
    }
  }
}

template <typename T, int K>
__device__ __attribute__((always_inline)) inline void recur_rows_any(const BlockHdr* hdr, int p, int base, int n, int rows, const T* Cs, int cl,
                                      const T* Rs, int rl, const T* Arec, const T* Brec, T* Ap, T* Bp) {
  // KE = p rounded up to even (the flush reads whole groups of four columns:
  // an odd-sized KE leaves column KE untouched, so the zero fill covers it)
  if (p <= 2) recur_rows<T, K, 2>(hdr, p, base, n, rows, Cs, cl, Rs, rl, Arec, Brec, Ap, Bp);
  else if (p <= 4) recur_rows<T, K, 4>(hdr, p, base, n, rows, Cs, cl, Rs, rl, Arec, Brec, Ap, Bp);
  else if (p <= 6) recur_rows<T, K, 6>(hdr, p, base, n, rows, Cs, cl, Rs, rl, Arec, Brec, Ap, Bp);
  else if (p <= 8) recur_rows<T, K, 8>(hdr, p, base, n, rows, Cs, cl, Rs, rl, Arec, Brec, Ap, Bp);
  else if (p <= 10) recur_rows<T, K, 10>(hdr, p, base, n, rows, Cs, cl, Rs, rl, Arec, Brec, Ap, Bp);
  else if (p <= 12) recur_rows<T, K, 12>(hdr, p, base, n, rows, Cs, cl, Rs, rl, Arec, Brec, Ap, Bp);
  else if (p <= 14) recur_rows<T, K, 14>(hdr, p, base, n, rows, Cs, cl, Rs, rl, Arec, Brec, Ap, Bp);
  else if (p <= 16) recur_rows<T, K, 16>(hdr, p, base, n, rows, Cs, cl, Rs, rl, Arec, Brec, Ap, Bp);
  else if constexpr (K > 16) {
    if (p <= 24) recur_rows<T, K, 24>(hdr, p, base, n, rows, Cs, cl, Rs, rl, Arec, Brec, Ap, Bp);
    else recur_rows<T, K, 32>(hdr, p, base, n, rows, Cs, cl, Rs, rl, Arec, Brec, Ap, Bp);
  }
}

// HOOKS: the decision log and tie-band replay of the tests (a separate
// instantiation, so that the plain sweep carries none of their work)
template <typename T, int K, int NT, bool HOOKS>
__global__ __launch_bounds__(256) void local_regs_kernel(LocalArgs a) {
  static_assert(K == 16 || K == 32, "blocks of whole tiles");
  extern __shared__ __align__(16) unsigned char smem[];
  typedef RegLds<T, K, NT> Lay;
  constexpr int KL = Lay::KL, P = Lay::P;
  constexpr int H = RegTiles<T, NT>::H;
  const int n = a.n, L = a.L, s = a.slice;
  const int np = pad16(n), nt = np / 16;
  const int cl = K + 1, rl = P + 1;
  const int c = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = uniform(tid >> 6);      // scalar: tile tests below become scalar branches
  const bool walker = wave == 0;
  const int wr = wave & 1, wc = wave >> 1;

  BlockHdr* hdr = (BlockHdr*)smem;
  SiteConst* sc = (SiteConst*)(smem + Lay::sc());
  uint8_t* rp = smem + Lay::rp(n);
  uint8_t* flags = smem + Lay::flags(n);
  double* Rv = (double*)(smem + Lay::rv(n));
  T* Ap = (T*)(smem + Lay::ap(n));         // [P][KL]: A
  T* Bp = (T*)(smem + Lay::bp(n));         // [P][KL]: Bv
  T* Cs = (T*)(smem + Lay::cs(n));         // [P][K+1]
  T* Rs = (T*)(smem + Lay::rs(n));         // [K][P+1]
  T* Arec = (T*)(smem + Lay::ar(n));       // [K][KR]: A[base + k, m]
  T* Brec = (T*)(smem + Lay::br(n));       // [K][KR]: Bv[base + k, m]

  // G into the accumulators
  RegTiles<T, NT> G;
  {
    const int nn = opaque(n);
    const T* Gg = (const T*)a.G + (long)c * nn * nn;
#pragma unroll
    for (int ta = 0; ta < H; ++ta)
#pragma unroll
      for (int tb = 0; tb < H; ++tb) {
        const int ti = wr + 2 * ta, tj = wc + 2 * tb;
        const int cc = tj * 16 + (lane & 15);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = ti * 16 + frag_row<T>(lane, v);
          G.t[ta][tb][v] = (r < nn && cc < nn) ? Gg[r * nn + cc] : T(0);
        }
      }
  }
  site_constants(a, c, sc, rp, flags, Rv);
  // strip rows and columns past N stay zero
  for (int e = tid; e < P * cl; e += blockDim.x) Cs[e] = T(0);
  for (int e = tid; e < K * rl; e += blockDim.x) Rs[e] = T(0);
  __syncthreads();

  // columns and rows [base, base + K) of G into Cs and Rs.  K is a multiple
  // of 16 and base of K, so the block is K / 16 whole tile columns (rows).
  // Tile column t is in this wave's grid iff t - wc is even, as its index
  // tb = (t - wc) / 2: one uniform test per tile column and row of the grid.
  auto extract = [&](int base) {
#pragma unroll
    for (int u = 0; u < K / 16; ++u) {
      const int t = (base >> 4) + u;
      const int tbr = ((t - wc) & 1) == 0 && t < nt ? (t - wc) >> 1 : -1;
      const int tar = ((t - wr) & 1) == 0 && t < nt ? (t - wr) >> 1 : -1;
      const int cc = t * 16 + (lane & 15) - base;
#pragma unroll
      for (int tb = 0; tb < H; ++tb) {
        if (tb == tbr) {
#pragma unroll
          for (int ta = 0; ta < H; ++ta) {
            const int ti = wr + 2 * ta;
            if (ti < nt) {
#pragma unroll
              for (int v = 0; v < 4; ++v) Cs[(ti * 16 + frag_row<T>(lane, v)) * cl + cc] = G.t[ta][tb][v];
            }
          }
        }
      }
#pragma unroll
      for (int ta = 0; ta < H; ++ta) {
        if (ta == tar) {
#pragma unroll
          for (int tb = 0; tb < H; ++tb) {
            const int tj = wc + 2 * tb;
            if (tj < nt) {
              const int c2 = tj * 16 + (lane & 15);
#pragma unroll
              for (int v = 0; v < 4; ++v) Rs[(t * 16 + frag_row<T>(lane, v) - base) * rl + c2] = G.t[ta][tb][v];
            }
          }
        }
      }
    }
  };
  extract(0);
  __syncthreads();

  const double band_lo = exp(-a.band), band_hi = exp(a.band);
  WalkState st = {0.0, 0, {0, 0}};
  for (int base = 0, blk = 0; base < n; base += K, ++blk) {
    if (walker) {
      auto g0 = [&](int r, int cc) { return Cs[(base + r) * cl + cc]; };
      if constexpr (K == 16)
        walk_dense<T, HOOKS>(g0, base, min(K, n - base), blk, sc, rp, hdr, Arec, Brec, flags, Rv, band_lo, band_hi,
                             st);
      else
        walk_diag<T, K, HOOKS>(g0, base, min(K, n - base), blk, sc, rp, hdr, Arec, Brec, flags, Rv, band_lo,
                               band_hi, st);
    }
    __syncthreads();
    const int p = hdr->p[blk & 1];
    if (p > 0) {                           // the same for every thread
      recur_rows_any<T, K>(hdr, p, base, n, P, Cs, cl, Rs, rl, Arec, Brec, Ap, Bp);
      __syncthreads();
      // G -= A Bv^T on the accumulators.  Every tile of the wave's grid is
      // multiplied, also those past nt: their rows of A and Bv lie in the
      // zero rows of the panels (tile rows < 32 H = P), so they stay zero
      // and are never stored; the MFMA chain then has no branches.
      const int mm = (p + 3) & ~3;
      for (int k0 = 0; k0 < mm; k0 += 4) {
        const int kk = k0 + (lane >> 4);
        T av[H], bv[H];
#pragma unroll
        for (int ta = 0; ta < H; ++ta) av[ta] = -Ap[((wr + 2 * ta) * 16 + (lane & 15)) * KL + kk];
#pragma unroll
        for (int tb = 0; tb < H; ++tb) bv[tb] = Bp[((wc + 2 * tb) * 16 + (lane & 15)) * KL + kk];
#pragma unroll
        for (int ta = 0; ta < H; ++ta)
#pragma unroll
          for (int tb = 0; tb < H; ++tb) G.t[ta][tb] = mfma16(av[ta], bv[tb], G.t[ta][tb]);
      }
    }
    if (base + K < n) extract(base + K);
    __syncthreads();
  }

  // fields, logs, counters; G back to global memory
  double* x = a.x + (long)c * L * n;
  for (int j = tid; j < n; j += blockDim.x) {
    const bool acc = flags[j] != 0;
    if (acc) x[s * n + j] = x[s * n + j] + sc[j].d;
    if (a.log_margin) {
      const long o = (long)c * L * n + s * n + j;
      a.log_margin[o] = (float)(log(sc[j].u) - log(Rv[j]));
      a.log_accept[o] = (uint8_t)acc;
    }
  }
  {
    const int nn = opaque(n);
    T* Gg = (T*)a.G + (long)c * nn * nn;
#pragma unroll
    for (int ta = 0; ta < H; ++ta)
#pragma unroll
      for (int tb = 0; tb < H; ++tb) {
        const int ti = wr + 2 * ta, tj = wc + 2 * tb;
        const int cc = tj * 16 + (lane & 15);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = ti * 16 + frag_row<T>(lane, v);
          if (r < nn && cc < nn) Gg[r * nn + cc] = G.t[ta][tb][v];
        }
      }
  }
  if (walker && lane == 0) {
    a.logdet[c] += st.logr;
    int64_t* cnt = a.counters + (long)c * N_COUNTERS;
    cnt[CNT_LOCAL_P] += n;
    cnt[CNT_LOCAL_A] += st.nacc;
    if (a.replay_counts) {
      a.replay_counts[2 * c] += st.counts[0];
      a.replay_counts[2 * c + 1] += st.counts[1];
    }
  }
}

// ===========================================================================
// streamed form: G in global memory
// ===========================================================================
// row stride (elements) of the A and Bv panels: 16-byte aligned rows
template <typename T, int K> struct Panel { enum { ld = K + 16 / (int)sizeof(T) }; };

template <typename T, int K>
struct StreamLds {
  static __host__ __device__ size_t sc() { return align16(sizeof(BlockHdr)); }
  static __host__ __device__ size_t rp(int n) { return sc() + sizeof(SiteConst) * (size_t)n; }
  static __host__ __device__ size_t flags(int n) { return rp(n) + n; }
  static __host__ __device__ size_t rv(int n) { return align16(flags(n) + n); }
  static __host__ __device__ size_t small(int n) { return align16(rv(n) + 8 * (size_t)n); }
  static __host__ __device__ size_t am(int n) { return small(n) + 4 * sizeof(T) * K * K; }
  static __host__ __device__ size_t bm(int n) { return am(n) + sizeof(T) * (size_t)pad16(n) * Panel<T, K>::ld; }
  static __host__ __device__ size_t total(int n) {
    return align16(bm(n) + sizeof(T) * (size_t)pad16(n) * Panel<T, K>::ld);
  }
};

// G <- G - A Bv^T over the first p columns, G global (row stride n); each
// wave takes TB tiles at a time so that their loads are in flight together
template <typename T, int K, int TB>
__device__ inline void flush_global(T* G, const T* Am, const T* Bm, int n, int np, int p) {
  constexpr int KL = Panel<T, K>::ld;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  typedef typename Frag<T>::type F;
  const int nt = np / 16, tiles = nt * nt;
  const int mm = (p + 3) & ~3;
  for (int t0 = wave * TB; t0 < tiles; t0 += 4 * TB) {
    F acc[TB];
    int ti[TB], tj[TB];
#pragma unroll
    for (int u = 0; u < TB; ++u) {
      const int t = min(t0 + u, tiles - 1);
      ti[u] = t / nt;
      tj[u] = t - ti[u] * nt;
      const int cc = tj[u] * 16 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = ti[u] * 16 + frag_row<T>(lane, v);
        acc[u][v] = (r < n && cc < n) ? G[r * n + cc] : T(0);
      }
    }
    for (int k0 = 0; k0 < mm; k0 += 4) {
#pragma unroll
      for (int u = 0; u < TB; ++u) {
        const T av = -Am[(ti[u] * 16 + (lane & 15)) * KL + k0 + (lane >> 4)];
        const T bv = Bm[(tj[u] * 16 + (lane & 15)) * KL + k0 + (lane >> 4)];
        acc[u] = mfma16(av, bv, acc[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < TB; ++u) {
      if (t0 + u >= tiles) break;
      const int cc = tj[u] * 16 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = ti[u] * 16 + frag_row<T>(lane, v);
        if (r < n && cc < n) G[r * n + cc] = acc[u][v];
      }
    }
  }
}

template <typename T, int K, int KE>
__device__ inline void recur_all_stream(const BlockHdr* hdr, const T* G, T* Am, T* Bm, const T* ASm, const T* BSm,
                                        int n, int np, int p) {
  constexpr int KL = Panel<T, K>::ld;
  const int npa = (np + 63) & ~63;         // A tasks fill whole waves, so isA is wave-uniform
  for (int t = threadIdx.x; t < 2 * npa; t += blockDim.x) {
    const bool isA = t < npa;
    const int j = isA ? t : t - npa;
    if (j >= np) continue;
    const bool live = j < n;
    const int jj = live ? j : 0;
    T g[KE];
#pragma unroll
    for (int mq = 0; mq < KE; ++mq) {
      const int im = uniform_site(hdr, mq, p);
      g[mq] = isA ? G[jj * n + im] : G[im * n + jj];
    }
    T v[KE];
    recur_row<T, K, KE>(hdr, p, isA, live, j, g, isA ? BSm : ASm, v);
    T* dst = (isA ? Am : Bm) + j * KL;
#pragma unroll
    for (int mq = 0; mq < KE; ++mq) dst[mq] = v[mq];
  }
}

template <typename T, int K>
__global__ __launch_bounds__(256) void local_stream_kernel(LocalArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  typedef StreamLds<T, K> Lay;
  const int n = a.n, L = a.L, s = a.slice;
  const int np = pad16(n);
  const int c = blockIdx.x;
  const int tid = threadIdx.x, wave = uniform(tid >> 6);

  BlockHdr* hdr = (BlockHdr*)smem;
  SiteConst* sc = (SiteConst*)(smem + Lay::sc());
  uint8_t* rp = smem + Lay::rp(n);
  uint8_t* flags = smem + Lay::flags(n);
  double* Rv = (double*)(smem + Lay::rv(n));
  T* As = (T*)(smem + Lay::small(n));
  T* Bs = As + K * K;
  T* ASm = Bs + K * K;
  T* BSm = ASm + K * K;
  T* Am = (T*)(smem + Lay::am(n));         // [np][KL] rows of A and Bv (entries >= p zero)
  T* Bm = (T*)(smem + Lay::bm(n));
  T* G = (T*)a.G + (long)c * n * n;

  site_constants(a, c, sc, rp, flags, Rv);
  for (int e = tid; e < 2 * np * Panel<T, K>::ld; e += 256) Am[e] = T(0);
  __syncthreads();

  const bool test_hooks = a.log_margin != nullptr || a.replay != nullptr;
  const double band_lo = exp(-a.band), band_hi = exp(a.band);
  WalkState st = {0.0, 0, {0, 0}};
  for (int base = 0, blk = 0; base < n; base += K, ++blk) {
    const int cnt = min(K, n - base);
    if (wave == 0)
      walk_block<T, K>([&](int r, int cc) { return G[(base + r) * n + base + cc]; }, base, cnt, blk, sc, rp, hdr, As,
                       Bs, flags, Rv, test_hooks, band_lo, band_hi, st);
    __syncthreads();
    const int p = hdr->p[blk & 1];
    if (p == 0) continue;                  // the same for every thread: nothing to flush
    gather_small<T, K>(hdr, As, Bs, ASm, BSm, base, p);
    __syncthreads();
    if (p <= 8) recur_all_stream<T, K, 8>(hdr, G, Am, Bm, ASm, BSm, n, np, p);
    else if (p <= 16) recur_all_stream<T, K, (K >= 16 ? 16 : 8)>(hdr, G, Am, Bm, ASm, BSm, n, np, p);
    else recur_all_stream<T, K, (K >= 32 ? 32 : 8)>(hdr, G, Am, Bm, ASm, BSm, n, np, p);
    __syncthreads();
    flush_global<T, K, 8>(G, Am, Bm, n, np, p);
    __syncthreads();
  }

  double* x = a.x + (long)c * L * n;
  for (int j = tid; j < n; j += 256) {
    const bool acc = flags[j] != 0;
    if (acc) x[s * n + j] = x[s * n + j] + sc[j].d;
    if (a.log_margin) {
      const long o = (long)c * L * n + s * n + j;
      a.log_margin[o] = (float)(log(sc[j].u) - log(Rv[j]));
      a.log_accept[o] = (uint8_t)acc;
    }
  }
  if (tid == 0) {
    a.logdet[c] += st.logr;
    int64_t* cnt = a.counters + (long)c * N_COUNTERS;
    cnt[CNT_LOCAL_P] += n;
    cnt[CNT_LOCAL_A] += st.nacc;
    if (a.replay_counts) {
      a.replay_counts[2 * c] += st.counts[0];
      a.replay_counts[2 * c + 1] += st.counts[1];
    }
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static const size_t kMaxLds = 160 * 1024;

// tile-grid classes of the register form: N <= 16 * NT.  Up to N = 144 the
// tiles and the walker's strips fit the register file with room to spare;
// an FP32 G of N = 256 fills the accumulators (64 tiles a wave) and the
// walker spills some of its strips, which still beats streaming G from
// memory.  FP64 beyond N = 144 takes the streamed form.
static int reg_class(int n, int precision) {
  const int nt = pad16(n) / 16;
  if (nt <= 4) return 4;
  if (nt <= 7) return 7;
  if (nt <= 9) return 9;
  if (nt <= 16 && precision) return 16;
  return 0;
}

template <typename T, int K>
static size_t lds_regs(int n, int rc) {
  switch (rc) {
    case 4: return RegLds<T, K, 4>::total(n);
    case 7: return RegLds<T, K, 7>::total(n);
    case 9: return RegLds<T, K, 9>::total(n);
    case 16: return RegLds<T, K, 16>::total(n);
    default: return ~(size_t)0;
  }
}
template <typename T, int K>
static size_t lds_t(int n, bool regs) {
  return regs ? lds_regs<T, K>(n, reg_class(n, sizeof(T) == 4)) : StreamLds<T, K>::total(n);
}

static bool use_regs(int n, int precision, int kd) {
  if (kd != 16 && kd != 32) return false;
  const int rc = reg_class(n, precision);
  if (!rc || (rc == 16 && kd != 16)) return false;   // N > 144: blocks of 16 only
  const size_t b = precision ? (kd == 16 ? lds_regs<float, 16>(n, rc) : lds_regs<float, 32>(n, rc))
                             : (kd == 16 ? lds_regs<double, 16>(n, rc) : lds_regs<double, 32>(n, rc));
  return b <= kMaxLds;
}

size_t local_lds_bytes(int n, int precision, int nt, int kd) {
  (void)nt;
  const bool r = use_regs(n, precision, kd);
  if (precision) return kd == 8 ? lds_t<float, 8>(n, r) : kd == 16 ? lds_t<float, 16>(n, r) : lds_t<float, 32>(n, r);
  return kd == 8 ? lds_t<double, 8>(n, r) : kd == 16 ? lds_t<double, 16>(n, r) : lds_t<double, 32>(n, r);
}

bool local_supported(int n, int precision, int nt, int kd) {
  if (n < 1 || n > 256 || (kd != 8 && kd != 16 && kd != 32)) return false;
  return local_lds_bytes(n, precision, nt, kd) <= kMaxLds;
}

bool local_g_in_lds(int n, int precision, int kd) { return use_regs(n, precision, kd); }

template <typename T, int K, int NT>
static hipError_t launch_regs(const LocalArgs& a, int chains, hipStream_t s) {
  const size_t lds = RegLds<T, K, NT>::total(a.n);
  if (a.log_margin != nullptr || a.replay != nullptr)
    hipLaunchKernelGGL((local_regs_kernel<T, K, NT, true>), dim3(chains), dim3(256), lds, s, a);
  else
    hipLaunchKernelGGL((local_regs_kernel<T, K, NT, false>), dim3(chains), dim3(256), lds, s, a);
  return hipGetLastError();
}

template <typename T, int K>
static hipError_t launch_k(const LocalArgs& a, int precision, int chains, hipStream_t s) {
  if constexpr (K == 16 || K == 32) {
    if (use_regs(a.n, precision, K)) {
      switch (reg_class(a.n, precision)) {
        case 4: return launch_regs<T, K, 4>(a, chains, s);
        case 7: return launch_regs<T, K, 7>(a, chains, s);
        case 9: return launch_regs<T, K, 9>(a, chains, s);
        case 16:
          if constexpr (sizeof(T) == 4 && K == 16) return launch_regs<T, K, 16>(a, chains, s);
          break;
        default: break;
      }
      return hipErrorInvalidValue;
    }
  }
  const size_t lds = StreamLds<T, K>::total(a.n);
  hipLaunchKernelGGL((local_stream_kernel<T, K>), dim3(chains), dim3(256), lds, s, a);
  return hipGetLastError();
}

template <typename F>
static hipError_t allow(F* f) {
  return hipFuncSetAttribute((const void*)f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxLds);
}

template <typename T>
static hipError_t allow_all_t() {
  hipError_t e = hipSuccess, x;
#define HQ_ALLOW(...)                  \
  x = allow(__VA_ARGS__);              \
  if (x != hipSuccess) e = x;
  HQ_ALLOW(local_stream_kernel<T, 8>);
  HQ_ALLOW(local_stream_kernel<T, 16>);
  HQ_ALLOW(local_stream_kernel<T, 32>);
  HQ_ALLOW(local_regs_kernel<T, 16, 4, false>);
  HQ_ALLOW(local_regs_kernel<T, 16, 4, true>);
  HQ_ALLOW(local_regs_kernel<T, 16, 7, false>);
  HQ_ALLOW(local_regs_kernel<T, 16, 7, true>);
  HQ_ALLOW(local_regs_kernel<T, 16, 9, false>);
  HQ_ALLOW(local_regs_kernel<T, 16, 9, true>);
  HQ_ALLOW(local_regs_kernel<T, 32, 4, false>);
  HQ_ALLOW(local_regs_kernel<T, 32, 4, true>);
  HQ_ALLOW(local_regs_kernel<T, 32, 7, false>);
  HQ_ALLOW(local_regs_kernel<T, 32, 7, true>);
  HQ_ALLOW(local_regs_kernel<T, 32, 9, false>);
  HQ_ALLOW(local_regs_kernel<T, 32, 9, true>);
  if constexpr (sizeof(T) == 4) {
    HQ_ALLOW(local_regs_kernel<T, 16, 16, false>);
    HQ_ALLOW(local_regs_kernel<T, 16, 16, true>);
  }
#undef HQ_ALLOW
  return e;
}

// raise the dynamic-LDS limit of every instantiation once, before any capture
hipError_t prepare_local() {
  const hipError_t e1 = allow_all_t<double>();
  const hipError_t e2 = allow_all_t<float>();
  return e1 != hipSuccess ? e1 : e2;
}

hipError_t launch_local(const LocalArgs& a, int precision, int nt, int kd, int chains, hipStream_t s) {
  if (!local_supported(a.n, precision, nt, kd)) return hipErrorInvalidValue;
  if (precision) {
    if (kd == 8) return launch_k<float, 8>(a, precision, chains, s);
    if (kd == 16) return launch_k<float, 16>(a, precision, chains, s);
    return launch_k<float, 32>(a, precision, chains, s);
  }
  if (kd == 8) return launch_k<double, 8>(a, precision, chains, s);
  if (kd == 16) return launch_k<double, 16>(a, precision, chains, s);
  return launch_k<double, 32>(a, precision, chains, s);
}

}  // namespace hq
